/* The 2D stage kernel (its own translation unit: it keeps the constant
 * table of the reconstruction in LDS, see mr_device.h, and is compiled
 * with its own scheduling options, see build.py). */
#define MR_KT_IN_LDS 1
#include "mr_common.h"

/* 2D stage kernel.  A work group owns a strip of CW = 256/NC consecutive
 * cells in x (two of them ring cells) and sweeps it upward over `rows` rows
 * plus one ring row below and one above.
 *
 * Moments (the strip plus two columns each side) sit in LDS rings: the cell
 * averages and y moments of rows y-2..y+2 (five rows: the modification of
 * the stencil's upper and lower cells reads rows y +- 2), the x moments of
 * rows y-1..y+1 (three rows); each value is loaded from HBM once per work
 * group, with the boundary condition applied when it is loaded, and the
 * rows needed next are fetched into registers while the current row is
 * computed.  Flags of rows y-1..y+1 sit in a three-row LDS ring.
 *
 * Stage 1 also writes the first moments of U^n after Step 2.2 (I.unm), which
 * the combination of stages 2 and 3 uses.
 *
 * With NC = 4 the four lanes of a cell each reconstruct one conserved
 * component, then each lane takes one row eta_r of the cell's 4x4
 * Gauss-Lobatto grid for the volume integrals, the left-face flux at eta_r
 * and the bottom-face flux at xi_r.  The top-face flux of a row is the
 * bottom-face flux of the next one, so the residual of row j is completed
 * while row j+1 is processed.  mode 0..2 = RK stage, 3 = write L(U).
 *
 * CH (characteristic-wise Step 1, NC = 4): lane k reconstructs field k of
 * the x set into the value slots, maps row eta_k of the cell back to the
 * conserved variables (R), takes the x-flux volume integral of that row
 * and the left-face flux; then the same with the y set for the y-flux
 * volume integral and the bottom-face flux, whose top traces the ring
 * keeps.  The moment rows of the next step are stored once both sets have
 * read the stencil. */
template <int NC>
struct mr2_lds {
  static constexpr int CW = MR_BLOCK / NC;   /* strip cells incl. ring */
  static constexpr int XW = CW + 4;          /* staged columns */
  static constexpr int NP = 3 * NC;          /* staged planes per row step */
  /* point-major layouts with padded strides: the lanes of one access
     (cells cs, roles/components k) fall on distinct LDS banks */
  static constexpr int CS = CW + 4;          /* component stride */
  static constexpr int VS = NC * CS + 1;     /* point stride of val */
  static constexpr int TS = NC * CS + 4;     /* point stride of top */
  static constexpr int FS = NC * CS;         /* stride of fs */
  /* plane strides chosen by measured LDS bank conflicts (mA padded by 2) */
  static constexpr int XP = XW + 2;
  double mA[5][2 * NC][XP];   /* planes (c, m = 0) and (c, m = 2): index 2c, 2c+1 */
  double mB[3][NC][XW];       /* planes (c, m = 1)                               */
  unsigned char flg[3][XW];
  double val[16 * VS];
  double top[4 * TS];
  double fs[2 * FS];
};

MR_INL int mr_mod3(int y) { return ((y % 3) + 3) % 3; }
MR_INL int mr_mod5(int y) { return ((y % 5) + 5) % 5; }

/* staged element e of a row step at row y (A planes at row y+1, B planes
   at row y): plane pl < 2 NC is A plane pl, else B plane pl - 2 NC */
template <int NC, int XW, bool STEP>
MR_INL double mr2_stage_ld(const mr_grid& g, int e, int xs0, int y) {
  const int pl = e / XW, col = e % XW;
  if (pl < 2 * NC) return mr_ld<STEP>(g, pl / 2, (pl % 2) * 2, xs0 + col, y + 1);
  return mr_ld<STEP>(g, pl - 2 * NC, 1, xs0 + col, y);
}

/* Characteristic-wise Step 1 (see mr_char2): field k of direction D of the
   cell at staged column c0, projected from the stencil in the LDS rings
   (the troubled cells' first moments modified when the cell is troubled)
   and reconstructed. */
template <bool BP, int D>
MR_INL void mr2_stage_field(const mr2_lds<4>& sh, const int* ra, const int* rb, const int* fs, int c0, int k,
                            const mr_char2& e, const mr_wconst& W, double val[16]) {
  double lk[4];
  mr_char2_left<D>(e, k, lk);
  double u[9], v[9], w[9];
#pragma unroll
  for (int dy = 0; dy < 3; ++dy)
#pragma unroll
    for (int dx = 0; dx < 3; ++dx) {
      const int l = dx + 3 * dy, cc = c0 + dx - 1;
      double a = 0.0, b = 0.0, d = 0.0;
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        a += lk[c] * sh.mA[ra[dy + 1]][2 * c][cc];
        b += lk[c] * sh.mB[rb[dy]][c][cc];
        d += lk[c] * sh.mA[ra[dy + 1]][2 * c + 1][cc];
      }
      u[l] = a; v[l] = b; w[l] = d;
    }
  if (fs[4]) {
#pragma unroll
    for (int dy = 0; dy < 3; ++dy)
#pragma unroll
      for (int dx = 0; dx < 3; ++dx) {
        const int l = dx + 3 * dy, cc = c0 + dx - 1;
        if (!fs[l]) continue;
        double b = 0.0, d = 0.0;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          b += lk[c] * mr_modified_moment(sh.mA[ra[dy + 1]][2 * c][cc - 1], sh.mA[ra[dy + 1]][2 * c][cc + 1],
                                          sh.mB[rb[dy]][c][cc - 1], sh.mB[rb[dy]][c][cc + 1]);
          d += lk[c] * mr_modified_moment(sh.mA[ra[dy]][2 * c][cc], sh.mA[ra[dy + 2]][2 * c][cc],
                                          sh.mA[ra[dy]][2 * c + 1][cc], sh.mA[ra[dy + 2]][2 * c + 1][cc]);
        }
        v[l] = b; w[l] = d;
      }
  }
  mr_recon2d<BP>(u, v, w, W, val);
}

template <int NC, bool BP, int GB, bool CH>
__global__ __launch_bounds__(MR_BLOCK) MR_OCC void k2_stage(const mr_inst* __restrict__ insts, const mr_tile2* __restrict__ tiles, int ntiles, int mode) {
  mr_kt_fill();
  using S = mr2_lds<NC>;
  constexpr int CW = S::CW, XW = S::XW, NP = S::NP, CS = S::CS, VS = S::VS, TS = S::TS, FS = S::FS;
  constexpr int NE = (NP * XW + MR_BLOCK - 1) / MR_BLOCK;   /* staged values per thread per row */
  __shared__ S sh;
  const int tid = threadIdx.x;
  const int cs = tid / NC, k = tid % NC;
  const int comp = (NC == 1) ? 0 : k;
#define VAL(p, c, cell) sh.val[(p) * VS + (c) * CS + (cell)]
#define TOP(q, c, cell) sh.top[(q) * TS + (c) * CS + (cell)]
#define FSM(m, c, cell) sh.fs[(m) * FS + (c) * CS + (cell)]
  for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const mr_tile2 tl = tiles[t];
    const mr_inst& I = insts[tl.inst];
    if (mode < 3 && !I.active) continue;
    const int st = mode == 3 ? 0 : mode;
    const mr_grid g{mr_gp(I.p_in[st]), I.plane, I.nx, I.ny, I.bcx, I.bcy, 3, GB ? &I : nullptr, mr_stage_time(I, mode)};
    const mr_grid gn{mr_gp(I.p_un), I.plane, I.nx, I.ny, I.bcx, I.bcy, 3, GB ? &I : nullptr, mr_stage_time(I, 0)};
    const MR_GLB unsigned char* fl = mr_gp(I.flags[(mode == 0 || mode == 3) ? 0 : 1]);
    MR_GLB double* unm = mr_gp(I.unm);
    const double rdx = I.rdx, rdy = I.rdy, dt = I.dt, gam = I.gam;
    const double alpha = (NC == 1) ? mr_bitsd(I.lfa[st]) : 0.0;
    MR_GLB double* O = mr_gp(I.p_out[st]);
    const long long P = I.plane;
    const int xs0 = tl.x0 - 3;                 /* strip column 0 */
    const int x = tl.x0 - 1 + cs;
    const bool outx = cs >= 1 && cs <= CW - 2 && x < I.nx;
    /* staged element q of this thread in every row step: plane and folded
       column as one element offset (A planes: bit 30 set); whether it is a
       first moment of a transmissive x ghost (reads as zero) or flips sign
       as a reflective x ghost; whether it is a first moment, and whether it
       flips in a reflective y ghost row */
    int soff[NE];
    unsigned szero = 0u, sfm = 0u, sneg = 0u, syflip = 0u;
#pragma unroll
    for (int q = 0; q < NE; ++q) {
      const int e = min(tid + q * MR_BLOCK, NP * XW - 1);
      const int pl = e / XW, col = e % XW;
      const bool isA = pl < 2 * NC;
      const int c = isA ? pl / 2 : pl - 2 * NC, m = isA ? (pl % 2) * 2 : 1;
      int kx = 0;
      const int ii = mr_fold(xs0 + col, I.nx, I.bcx, &kx);
      soff[q] = ((c * 3 + m) * (int)P + ii) | (isA ? (1 << 30) : 0);
      if (m != 0) sfm |= 1u << q;
      if (m != 0 && kx == 1) szero |= 1u << q;
      if (kx == 2 && mr_refl_flip(c, m, 0)) sneg |= 1u << q;
      if (mr_refl_flip(c, m, 1)) syflip |= 1u << q;
    }
    /* ---- prologue: A rows y0-3 .. y0+1, B and flag rows y0-2 .. y0 ---- */
    for (int r = tl.y0 - 3; r <= tl.y0 - 2; ++r)
      for (int e = tid; e < 2 * NC * XW; e += MR_BLOCK)
        sh.mA[mr_mod5(r)][e / XW][e % XW] = mr_ld<GB == 2>(g, (e / XW) / 2, ((e / XW) % 2) * 2, xs0 + e % XW, r);
    for (int r = tl.y0 - 2; r <= tl.y0; ++r) {
      for (int e = tid; e < NP * XW; e += MR_BLOCK) {
        const double v = mr2_stage_ld<NC, XW, GB == 2>(g, e, xs0, r);
        if (e / XW < 2 * NC) sh.mA[mr_mod5(r + 1)][e / XW][e % XW] = v;
        else sh.mB[mr_mod3(r)][e / XW - 2 * NC][e % XW] = v;
      }
      for (int e = tid; e < XW; e += MR_BLOCK)
        sh.flg[mr_mod3(r)][e] = (unsigned char)mr_flag(fl, I.fex, I.fey, I.fhalo, xs0 + e, r);
    }
    __syncthreads();
    double pAu = 0.0, pAv = 0.0, pAw = 0.0, pB0 = 0.0, pB1 = 0.0, pU = 0.0, pV = 0.0, pW = 0.0;
    for (int jr = -1; jr <= tl.rows; ++jr) {
      const int y = tl.y0 + jr;
      /* stages 2 and 3: U^n of the row finished in this step, loaded now so
         that the latency hides behind the reconstruction */
      double qun = 0.0, qvn = 0.0, qwn = 0.0;
      if ((mode == 1 || mode == 2) && jr >= 1 && outx) {
        const long long cell = (long long)(y - 1) * I.nx + x;
        const MR_GLB double* vs = I.mod == 0 ? unm + (long long)(comp * 2) * P : gn.U + (long long)(comp * 3 + 1) * P;
        qun = gn.U[(long long)(comp * 3) * P + cell];
        qvn = vs[cell];
        qwn = vs[P + cell];
      }
      /* prefetch A row y+3, B and flag row y+2 (stored once rows y-2 and
         y-1 are consumed) */
      double pre[NE];
      unsigned pzero = 0u, pneg = 0u;   /* elements that read as zero / flip (applied when stored) */
      unsigned char pref = 0;
      {
        /* row folds are uniform over the work group */
        int kA = 0, kB = 0;
        const int jA = mr_fold(y + 3, I.ny, I.bcy, &kA) * I.nx;
        const int jB = mr_fold(y + 2, I.ny, I.bcy, &kB) * I.nx;
#pragma unroll
        for (int q = 0; q < NE; ++q) {
          const int o = soff[q];
          const bool isA = (o >> 30) & 1;
          const int off = (o & ((1 << 30) - 1)) + (isA ? jA : jB);
          pre[q] = g.U[off];
          const int ky = isA ? kA : kB;
          /* first moments of transmissive ghosts are zero; reflective ghosts
             flip the moments mr_refl_flip names */
          if (((szero >> q) & 1u) || (((sfm >> q) & 1u) && ky == 1)) pzero |= 1u << q;
          if (((sneg >> q) & 1u) != (ky == 2 && ((syflip >> q) & 1u))) pneg |= 1u << q;
        }
      }
      if (tid < XW) pref = (unsigned char)mr_flag(fl, I.fex, I.fey, I.fhalo, xs0 + tid, y + 2);
      /* ---- Steps 1, 2.2, 2.3 for component `comp` of cell (x, y) ---- */
      double cu, cv, cw;
      /* characteristic-wise: the stencil rows, flags and the cell's state */
      int cra[5], crb[3], cfs[9];
      mr_char2 ex{}, ey{};
      if constexpr (CH) {
        const int c0 = cs + 2;
        for (int q = 0; q < 5; ++q) cra[q] = mr_mod5(y - 2 + q);
        for (int q = 0; q < 3; ++q) crb[q] = mr_mod3(y - 1 + q);
#pragma unroll
        for (int l = 0; l < 9; ++l) cfs[l] = sh.flg[crb[l / 3]][c0 + l % 3 - 1];
        double u0[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) u0[c] = sh.mA[cra[2]][2 * c][c0];
        ex = mr_char2_state<0>(u0, gam);
        ey = mr_char2_state<1>(u0, gam);
        cu = u0[comp];
        const bool md = cfs[4] && I.mod != 1;
        cv = md ? mr_modified_moment(sh.mA[cra[2]][2 * comp][c0 - 1], sh.mA[cra[2]][2 * comp][c0 + 1],
                                     sh.mB[crb[1]][comp][c0 - 1], sh.mB[crb[1]][comp][c0 + 1])
                : sh.mB[crb[1]][comp][c0];
        cw = md ? mr_modified_moment(sh.mA[cra[1]][2 * comp][c0], sh.mA[cra[3]][2 * comp][c0],
                                     sh.mA[cra[1]][2 * comp + 1][c0], sh.mA[cra[3]][2 * comp + 1][c0])
                : sh.mA[cra[2]][2 * comp + 1][c0];
        double val[16];
        mr2_stage_field<BP, 0>(sh, cra, crb, cfs, c0, comp, ex, I.W, val);
#pragma unroll
        for (int q = 0; q < 16; ++q) VAL(q, comp, cs) = val[q];
      } else {
        const int ra[5] = {mr_mod5(y - 2), mr_mod5(y - 1), mr_mod5(y), mr_mod5(y + 1), mr_mod5(y + 2)};
        const int rb[3] = {mr_mod3(y - 1), mr_mod3(y), mr_mod3(y + 1)};
        const int c0 = cs + 2;                    /* staged column of cell x */
        double u[9], v[9], w[9];
        int fs[9];
#pragma unroll
        for (int dy = 0; dy < 3; ++dy)
#pragma unroll
          for (int dx = 0; dx < 3; ++dx) {
            const int l = dx + 3 * dy;
            u[l] = sh.mA[ra[dy + 1]][2 * comp][c0 + dx - 1];
            v[l] = sh.mB[rb[dy]][comp][c0 + dx - 1];
            w[l] = sh.mA[ra[dy + 1]][2 * comp + 1][c0 + dx - 1];
            fs[l] = sh.flg[rb[dy]][c0 + dx - 1];
          }
        if (fs[4]) {
          /* troubled cell: first moments of the troubled cells of the
             stencil modified from the unmodified input (Jacobi) */
#pragma unroll
          for (int dy = 0; dy < 3; ++dy)
#pragma unroll
            for (int dx = 0; dx < 3; ++dx) {
              const int l = dx + 3 * dy;
              if (!fs[l]) continue;
              const int cc = c0 + dx - 1;
              v[l] = mr_modified_moment(sh.mA[ra[dy + 1]][2 * comp][cc - 1], sh.mA[ra[dy + 1]][2 * comp][cc + 1],
                                        sh.mB[rb[dy]][comp][cc - 1], sh.mB[rb[dy]][comp][cc + 1]);
              w[l] = mr_modified_moment(sh.mA[ra[dy]][2 * comp][cc], sh.mA[ra[dy + 2]][2 * comp][cc],
                                        sh.mA[ra[dy]][2 * comp + 1][cc], sh.mA[ra[dy + 2]][2 * comp + 1][cc]);
            }
        }
        cu = u[4];
        /* the combination takes the modified first moments unless the
           modification stays internal to L */
        cv = I.mod == 1 ? sh.mB[rb[1]][comp][c0] : v[4];
        cw = I.mod == 1 ? sh.mA[ra[2]][2 * comp + 1][c0] : w[4];
        double val[16];
        mr_recon2d<BP>(u, v, w, I.W, val);
#pragma unroll
        for (int q = 0; q < 16; ++q) VAL(q, comp, cs) = val[q];
      }
      __syncthreads();
      /* the slots of A row y-2 and of B/flag row y-1 are consumed: store
         A row y+3 and B/flag row y+2 */
      auto store_rows = [&]() {
        const int sa = mr_mod5(y + 3), sb = mr_mod3(y + 2);
#pragma unroll
        for (int q = 0; q < NE; ++q) {
          const int e = tid + q * MR_BLOCK;
          if (e < NP * XW) {
            const double v = ((pzero >> q) & 1u) ? 0.0 : (((pneg >> q) & 1u) ? -pre[q] : pre[q]);
            if (e / XW < 2 * NC) sh.mA[sa][e / XW][e % XW] = v;
            else sh.mB[sb][e / XW - 2 * NC][e % XW] = v;
          }
        }
        if (tid < XW) sh.flg[sb][tid] = pref;
        if (GB && mr_presc_rows<GB == 2>(I, xs0, XW, y + 2, 2)) {
          /* ghosts that hold prescribed data */
          const double tb = mr_stage_time(I, mode);
#pragma unroll 1
          for (int q = 0; q < NE; ++q) {
            const int e = tid + q * MR_BLOCK;
            if (e < NP * XW) {
              const int pl = e / XW, col = e % XW;
              const bool isA = pl < 2 * NC;
              const int c = isA ? pl / 2 : pl - 2 * NC, m = isA ? (pl % 2) * 2 : 1;
              double v;
              if (mr_presc(I, c, m, xs0 + col, isA ? y + 3 : y + 2, tb, &v) ||
                  (GB == 2 && mr_step_val(I, g.U, c, m, xs0 + col, isA ? y + 3 : y + 2, &v))) {
                if (isA) sh.mA[sa][pl][col] = v;
                else sh.mB[sb][pl - 2 * NC][col] = v;
              }
            }
          }
        }
      };
      /* ---- volume integrals and the fluxes this lane owns ---- */
      double F[NC], G[NC], XL0[NC], XL1[NC], YB0[NC], YB1[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) F[c] = G[c] = XL0[c] = XL1[c] = YB0[c] = YB1[c] = 0.0;
      const bool body = jr >= 0 && jr < tl.rows;
      if constexpr (CH) {
        /* lane k = row eta_k of the cell: x set back to conserved variables */
        const int r = k;
        const double wr = glw(r), er = gln(r);
        double pts[4][4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          double wq[4];
#pragma unroll
          for (int j = 0; j < 4; ++j) wq[j] = VAL(q + 4 * r, j, cs);
          mr_char2_right<0>(ex, wq, pts[q]);
        }
        /* row eta_k of the cell is read and written by lane k only */
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
          for (int c = 0; c < 4; ++c) VAL(q + 4 * r, c, cs) = pts[q][c];
        if (body) {
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            double f[4];
            mr_euler_flux<4, 0>(pts[q], gam, f);
            const double wq = glw(q) * wr;
#pragma unroll
            for (int c = 0; c < 4; ++c) F[c] += wq * f[c];
          }
        }
        __syncthreads();
        if (body && cs >= 1) {
          double a[4], fh[4];
#pragma unroll
          for (int c = 0; c < 4; ++c) a[c] = VAL(3 + 4 * r, c, cs - 1);
          mr_face_flux<4, 0, GB == 2>(I, a, pts[0], gam, alpha, x, y, mr_stage_time(I, mode), fh);
#pragma unroll
          for (int c = 0; c < 4; ++c) { XL0[c] += wr * fh[c]; XL1[c] += wr * er * fh[c]; }
        }
        __syncthreads();
        /* field k of the y set (the stencil rows are still in place) */
        {
          double val[16];
          mr2_stage_field<BP, 1>(sh, cra, crb, cfs, cs + 2, comp, ey, I.W, val);
#pragma unroll
          for (int q = 0; q < 16; ++q) VAL(q, comp, cs) = val[q];
        }
        __syncthreads();
        store_rows();
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          double wq[4];
#pragma unroll
          for (int j = 0; j < 4; ++j) wq[j] = VAL(q + 4 * r, j, cs);
          mr_char2_right<1>(ey, wq, pts[q]);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
          for (int c = 0; c < 4; ++c) VAL(q + 4 * r, c, cs) = pts[q][c];
        if (body) {
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            double g4[4];
            mr_euler_flux<4, 1>(pts[q], gam, g4);
            const double wq = glw(q) * wr;
#pragma unroll
            for (int c = 0; c < 4; ++c) G[c] += wq * g4[c];
          }
        }
        __syncthreads();
        if (jr >= 0) {
          double a[4], b[4], gh[4];
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            a[c] = TOP(r, c, cs);
            b[c] = VAL(r, c, cs);
          }
          mr_face_flux<4, 1, GB == 2>(I, a, b, gam, alpha, y, x, mr_stage_time(I, mode), gh);
#pragma unroll
          for (int c = 0; c < 4; ++c) { YB0[c] += wr * gh[c]; YB1[c] += wr * er * gh[c]; }
        }
      } else {
      store_rows();
#pragma unroll
      for (int rr = 0; rr < 4 / NC; ++rr) {
        const int r = (NC == 1) ? rr : k;
        const double wr = glw(r), er = gln(r);
        if (body) {
          double pts[4][NC], rr4[4];
#pragma unroll
          for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int c = 0; c < NC; ++c) pts[q][c] = VAL(q + 4 * r, c, cs);
          if (NC == 4) mr_recip4(pts[0][0], pts[1][0], pts[2][0], pts[3][0], rr4);
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            double f[NC], gg[NC];
            if (NC == 4) mr_euler_fg_r(pts[q], rr4[q], gam, f, gg);
            else { f[0] = 0.5 * pts[q][0] * pts[q][0]; gg[0] = f[0]; }
            const double wq = glw(q) * wr;
#pragma unroll
            for (int c = 0; c < NC; ++c) { F[c] += wq * f[c]; G[c] += wq * gg[c]; }
          }
          if (cs >= 1) {
            double a[NC], b[NC], fh[NC];
#pragma unroll
            for (int c = 0; c < NC; ++c) {
              a[c] = VAL(3 + 4 * r, c, cs - 1);
              b[c] = VAL(4 * r, c, cs);
            }
            mr_face_flux<NC, 0, GB == 2>(I, a, b, gam, alpha, x, y, mr_stage_time(I, mode), fh);
#pragma unroll
            for (int c = 0; c < NC; ++c) { XL0[c] += wr * fh[c]; XL1[c] += wr * er * fh[c]; }
          }
        }
        if (jr >= 0) {
          double a[NC], b[NC], gh[NC];
#pragma unroll
          for (int c = 0; c < NC; ++c) {
            a[c] = TOP(r, c, cs);
            b[c] = VAL(r, c, cs);
          }
          mr_face_flux<NC, 1, GB == 2>(I, a, b, gam, alpha, y, x, mr_stage_time(I, mode), gh);
#pragma unroll
          for (int c = 0; c < NC; ++c) { YB0[c] += wr * gh[c]; YB1[c] += wr * er * gh[c]; }
        }
      }
      }
      /* lane k collects component k's sums */
      const double fF = mr_rs<NC>(F, k), fG = mr_rs<NC>(G, k);
      const double xl0 = mr_rs<NC>(XL0, k), xl1 = mr_rs<NC>(XL1, k);
      const double yb0 = mr_rs<NC>(YB0, k), yb1 = mr_rs<NC>(YB1, k);
      FSM(0, comp, cs) = xl0;
      FSM(1, comp, cs) = xl1;
      __syncthreads();
      /* the row below has consumed its top trace; store this row's */
#pragma unroll
      for (int q = 0; q < 4; ++q) TOP(q, comp, cs) = VAL(12 + q, comp, cs);
      /* ---- finish the row below: its top face is this row's bottom face ---- */
      if (jr >= 1 && outx) {
        const int yp = y - 1;
        const double Lu = pAu - (yb0 - pB0) * rdy;
        const double Lv = pAv - (yb1 - pB1) * rdy;
        const double Lw = pAw - (yb0 + pB0) * (0.5 * rdy);
        double r0, r1, r2;
        const long long cell = (long long)yp * I.nx + x;
        if (mode == 3) { r0 = Lu; r1 = Lv; r2 = Lw; }
        else if (mode == 0) {
          r0 = pU + dt * Lu; r1 = pV + dt * Lv; r2 = pW + dt * Lw;
          /* U^n after Step 2.2 (its first moments) for stages 2 and 3 */
          if (I.mod == 0) {
            const bool sol = GB == 2 && mr_solid(I, x, yp);
            unm[(long long)(comp * 2 + 0) * P + cell] = sol ? 0.0 : pV;
            unm[(long long)(comp * 2 + 1) * P + cell] = sol ? 0.0 : pW;
          }
        } else {
          const double a = mode == 1 ? 0.75 : 1.0 / 3.0, b = mode == 1 ? 0.25 : 2.0 / 3.0;
          const double un = qun, vn = qvn, wn = qwn;
          r0 = a * un + b * pU + b * dt * Lu;
          r1 = a * vn + b * pV + b * dt * Lv;
          r2 = a * wn + b * pW + b * dt * Lw;
        }
        if (GB == 2 && mr_solid(I, x, yp)) r0 = r1 = r2 = 0.0;   /* the step's cells carry no state */
        O[(long long)(comp * 3 + 0) * P + cell] = r0;
        O[(long long)(comp * 3 + 1) * P + cell] = r1;
        O[(long long)(comp * 3 + 2) * P + cell] = r2;
      }
      /* ---- this row's partial residual (all but the top face) ---- */
      if (cs + 1 < CW) {
        const double xr0 = FSM(0, comp, cs + 1);
        const double xr1 = FSM(1, comp, cs + 1);
        pAu = -(xr0 - xl0) * rdx;
        pAv = -(xr0 + xl0) * (0.5 * rdx) + fF * rdx;
        pAw = -(xr1 - xl1) * rdx + fG * rdy;
      }
      pB0 = yb0;
      pB1 = yb1;
      pU = cu;
      pV = cv;
      pW = cw;
      __syncthreads();
    }
  }
#undef VAL
#undef TOP
#undef FSM
}

/* gb: 0 no instance of the list has per-side boundary data (the variant
   without that code), 1 some have ghosts that hold a prescribed state, 2
   some also have a step or the wall flux (Euler); ch: the
   characteristic-wise Step 1 (nc = 4) */
extern "C" hipError_t mr_launch_stage2(hipStream_t s, int nc, int bp, int gb, int ch, mr_inst* d, const mr_tile2* t,
                                       int nt, int mode, int grid) {
  if (nt <= 0) return hipSuccess;
  const dim3 G(grid > 0 && grid < nt ? grid : nt), B(MR_BLOCK);
#define MR_L2(NC_, BP_, CH_)                                                                           \
  do {                                                                                                 \
    if (gb == 2 && NC_ == 4) hipLaunchKernelGGL((k2_stage<NC_, BP_, 2, CH_>), G, B, 0, s, d, t, nt, mode); \
    else if (gb) hipLaunchKernelGGL((k2_stage<NC_, BP_, 1, CH_>), G, B, 0, s, d, t, nt, mode);         \
    else hipLaunchKernelGGL((k2_stage<NC_, BP_, 0, CH_>), G, B, 0, s, d, t, nt, mode);                 \
  } while (0)
  if (nc == 1) { if (bp) MR_L2(1, true, false); else MR_L2(1, false, false); }
  else if (nc == 4 && !ch) { if (bp) MR_L2(4, true, false); else MR_L2(4, false, false); }
  else if (nc == 4) { if (bp) MR_L2(4, true, true); else MR_L2(4, false, true); }
  else return hipErrorInvalidValue;
#undef MR_L2
  return hipGetLastError();
}
