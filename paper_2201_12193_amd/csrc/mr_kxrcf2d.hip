/* The fused 2D KXRCF / TVB indicator kernel (its own translation unit: it
 * keeps the constant table of the reconstruction in LDS, see mr_device.h). */
#define MR_KT_IN_LDS 1
#include "mr_common.h"

/* ========================================= fused KXRCF / TVB (2D, tc = 1 or 4) */
/* Troubled-cell flags of eq. (KXRCF_) with the face averages of eq.
 * (line-integral-average_), in one pass: a work group owns a strip of 62
 * flag columns and sweeps it upward four rows at a time.  Each thread
 * reconstructs one cell (Step 1 on the unmodified stage input) of the
 * strip plus one ring column each side and keeps its face data in LDS; once
 * the rows above and below are there, the flags of the strip's cells follow
 * from the face data of the cell and its four neighbours.
 *
 * Moments of the strip (64 + 2 columns, the planes the indicator reads) sit
 * in a ten-row LDS ring, each loaded from HBM once per work group with the
 * boundary condition applied: a step reads six rows and writes the four
 * that the next step adds.  The face data sit in a six-row ring. */
#define KX_W 64                       /* reconstructed columns of a strip */
#define KX_XW (KX_W + 2)              /* staged columns                   */
#define KX_MR 10                      /* moment ring rows                 */
#define KX_FR 6                       /* face data ring rows              */

/* ring slot of row y >= -12 */
MR_INL int kx_slot(int y, int n) { return (y + 12 * n) % n; }

/* face data of the cell at staged column col whose rows y-1, y, y+1 sit in
   ring slots s0, s1, s2 (f as mr2_face_summary; the velocities use shared
   reciprocals of the density at the twelve face points) */
template <int NK, bool BP>
MR_INL void kx_face_data(const double (*mom)[3 * NK * KX_XW], int s0, int s1, int s2, int col,
                         const mr_wconst& W, double tvb_mh2, double f[9]) {
  double irl[4], irr[4], irm[4];   /* 1/rho at points 0,4,8,12 | 3,7,11,15 | 1,2,13,14 */
  double sl = 0.0, sr = 0.0, sb = 0.0, st = 0.0, nrm = 0.0;
  double vl = 0.0, vr = 0.0, vb = 0.0, vt = 0.0;
#pragma unroll 1
  for (int c = 0; c < NK; ++c) {
    /* the constant table stays in LDS: no loads of it are hoisted out of
       the component loop (they would hold its entries in registers) */
    __asm__ volatile("" ::: "memory");
    double u[9], v[9], w[9], q[16];
#pragma unroll
    for (int l = 0; l < 9; ++l) {
      const int dx = l % 3 - 1, slot = l < 3 ? s0 : (l < 6 ? s1 : s2);
      u[l] = mom[slot][(3 * c + 0) * KX_XW + col + dx];
      v[l] = mom[slot][(3 * c + 1) * KX_XW + col + dx];
      w[l] = mom[slot][(3 * c + 2) * KX_XW + col + dx];
    }
    mr_recon2d<BP>(u, v, w, W, q);
    if (c == 0) {
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        sl += glw(m) * q[0 + 4 * m];
        sr += glw(m) * q[3 + 4 * m];
        sb += glw(m) * q[m];
        st += glw(m) * q[12 + m];
      }
#pragma unroll
      for (int k = 0; k < 16; ++k) nrm = fmax(nrm, fabs(q[k]));
      if (NK == 1) { vl = sl; vr = sr; vb = sb; vt = st; }   /* Burgers: f'(u) = u */
      if (NK == 1 && tvb_mh2 >= 0.0) {
        /* TVB minmod test on the face averages (x then y); the verdict goes
           in f[0] */
        const double dpx = u[5] - u[4], dmx = u[4] - u[3], dpy = u[7] - u[4], dmy = u[4] - u[1];
        sl = (mr_tvb_changes(sr - u[4], dpx, dmx, tvb_mh2) || mr_tvb_changes(u[4] - sl, dpx, dmx, tvb_mh2) ||
              mr_tvb_changes(st - u[4], dpy, dmy, tvb_mh2) || mr_tvb_changes(u[4] - sb, dpy, dmy, tvb_mh2))
                 ? 1.0 : 0.0;
      }
      if (NK > 1) {
        mr_recip4(q[0], q[4], q[8], q[12], irl);
        mr_recip4(q[3], q[7], q[11], q[15], irr);
        mr_recip4(q[1], q[2], q[13], q[14], irm);
      }
    } else if (c == 1) {
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        vl += glw(m) * (q[0 + 4 * m] * irl[m]);
        vr += glw(m) * (q[3 + 4 * m] * irr[m]);
      }
    } else {
      vb = glw(0) * (q[0] * irl[0]) + glw(1) * (q[1] * irm[0]) + glw(2) * (q[2] * irm[1]) + glw(3) * (q[3] * irr[0]);
      vt = glw(0) * (q[12] * irl[3]) + glw(1) * (q[13] * irm[2]) + glw(2) * (q[14] * irm[3]) + glw(3) * (q[15] * irr[3]);
    }
  }
  f[0] = sl; f[1] = sr; f[2] = sb; f[3] = st;
  f[4] = vl; f[5] = vr; f[6] = vb; f[7] = vt;
  f[8] = nrm;
}

/* face data of one direction D of the characteristic-wise Step 1 (2D
   Euler, four components staged; see mr_char2): each field projected from
   the stencil, reconstructed, and mapped back at the points the indicator
   reads -- the density at all sixteen points (its norm), the density and
   the normal momentum at the points of the two faces normal to D.
   f[0..1] / f[4..5] (D = 0: left, right) or f[2..3] / f[6..7] (D = 1:
   bottom, top) as kx_face_data; *nrm is raised to max |rho|. */
template <bool BP, int D>
MR_INL void kx_face_data_ch(const double (*mom)[3 * 4 * KX_XW], int s0, int s1, int s2, int col,
                            const mr_wconst& W, double gam, double f[9], double* nrm) {
  double u0[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) u0[c] = mom[s1][(3 * c + 0) * KX_XW + col];
  const mr_char2 e = mr_char2_state<D>(u0, gam);
  double rho[16], mn[8];
#pragma unroll
  for (int q = 0; q < 16; ++q) rho[q] = 0.0;
#pragma unroll
  for (int q = 0; q < 8; ++q) mn[q] = 0.0;
#pragma unroll 1
  for (int k = 0; k < 4; ++k) {
    __asm__ volatile("" ::: "memory");   /* keep the constant table in LDS (see kx_face_data) */
    double lk[4];
    mr_char2_left<D>(e, k, lk);
    double u[9], v[9], w[9], q[16];
#pragma unroll
    for (int l = 0; l < 9; ++l) {
      const int dx = l % 3 - 1, slot = l < 3 ? s0 : (l < 6 ? s1 : s2);
      u[l] = v[l] = w[l] = 0.0;
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        u[l] += lk[c] * mom[slot][(3 * c + 0) * KX_XW + col + dx];
        v[l] += lk[c] * mom[slot][(3 * c + 1) * KX_XW + col + dx];
        w[l] += lk[c] * mom[slot][(3 * c + 2) * KX_XW + col + dx];
      }
    }
    mr_recon2d<BP>(u, v, w, W, q);
    /* column k of R: density entry 1, 1, 0, 1; normal momentum vn - c, vn, 0, vn + c */
    const double rr = k == 2 ? 0.0 : 1.0;
    const double rn = k == 0 ? e.vn - e.c : (k == 1 ? e.vn : (k == 2 ? 0.0 : e.vn + e.c));
#pragma unroll
    for (int p = 0; p < 16; ++p) rho[p] += rr * q[p];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const int pa = D == 0 ? 4 * m : m, pb = D == 0 ? 3 + 4 * m : 12 + m;
      mn[m] += rn * q[pa];
      mn[4 + m] += rn * q[pb];
    }
  }
#pragma unroll
  for (int p = 0; p < 16; ++p) *nrm = fmax(*nrm, fabs(rho[p]));
  double sa = 0.0, sb = 0.0, va = 0.0, vb = 0.0;
  double ia[4], ib[4];
  if (D == 0) { mr_recip4(rho[0], rho[4], rho[8], rho[12], ia); mr_recip4(rho[3], rho[7], rho[11], rho[15], ib); }
  else { mr_recip4(rho[0], rho[1], rho[2], rho[3], ia); mr_recip4(rho[12], rho[13], rho[14], rho[15], ib); }
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    const int pa = D == 0 ? 4 * m : m, pb = D == 0 ? 3 + 4 * m : 12 + m;
    sa += glw(m) * rho[pa];
    sb += glw(m) * rho[pb];
    va += glw(m) * (mn[m] * ia[m]);
    vb += glw(m) * (mn[4 + m] * ib[m]);
  }
  f[2 * D] = sa; f[2 * D + 1] = sb;
  f[4 + 2 * D] = va; f[5 + 2 * D] = vb;
}

/* NK: components the indicator reads (1 Burgers, 3 Euler: rho and the
   momenta; 4 Euler with the characteristic-wise Step 1, whose fields mix
   all components; 1 for the TVB minmod test, which reads the indicator
   variable only and decides each cell from its own face averages).  Work item: flag columns x0 .. x0+61, flag rows y0 .. y0+rows-1
   of the extended flag range [-2, n+2)^2 (y0 >= -2). */
template <int NK, bool BP, int GB>
__global__ __launch_bounds__(MR_BLOCK) MR_OCC void k2_kxrcf(const mr_inst* __restrict__ insts, const mr_tile2* __restrict__ tiles, int ntiles, int stage) {
  mr_kt_fill();
  constexpr int NPL = 3 * NK;
  constexpr int NROW = NPL * KX_XW;                       /* staged values per row */
  constexpr int NQ = (NROW + MR_BLOCK - 1) / MR_BLOCK;    /* ... per thread        */
  __shared__ double mom[KX_MR][NROW];                     /* [row][plane][column]  */
  __shared__ double fd[KX_FR][9][KX_W];
  const int tid = threadIdx.x, cx = tid % KX_W, ry = tid / KX_W;
  for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const mr_tile2 tl = tiles[t];
    const mr_inst& I = insts[tl.inst];
    if (stage < 3 && !I.active) continue;
    const MR_GLB double* U = mr_gp(stage < 3 ? I.p_in[stage] : I.buf[0]);
    MR_GLB unsigned char* fl = mr_gp(I.flags[(stage == 0 || stage == 3) ? 0 : 1]);
    MR_GLB double* aleph = mr_gp(I.aleph);
    const int xs = tl.x0 - 2;              /* staged column 0 */
    const int ylast = tl.y0 + tl.rows;     /* last reconstructed row */
    const double tb = mr_stage_time(I, stage);
    /* staged element q of this thread in every row: plane offset plus folded
       column; whether it is a first moment (of a transmissive x ghost:
       zero), flips as a reflective x ghost, flips in a reflective y row */
    int soff[NQ];
    unsigned szero = 0u, sfm = 0u, sneg = 0u, syflip = 0u;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int e = min(tid + q * MR_BLOCK, NROW - 1);
      const int pl = e / KX_XW, c = pl / 3, m = pl % 3;
      int kx = 0;
      const int ii = mr_fold(xs + e % KX_XW, I.nx, I.bcx, &kx);
      soff[q] = pl * (int)I.plane + ii;
      if (m != 0) sfm |= 1u << q;
      if (m != 0 && kx == 1) szero |= 1u << q;
      if (kx == 2 && mr_refl_flip(c, m, 0)) sneg |= 1u << q;
      if (mr_refl_flip(c, m, 1)) syflip |= 1u << q;
    }
    /* fetch moment row y into v; the elements that read as zero (first
       moments of transmissive ghosts) are marked in the low bits of *z, the
       ones that flip sign (reflective ghosts) from bit 16, both applied when
       stored.  The fold of y is uniform over the work group. */
    auto fetch = [&](int y, double* v, unsigned* z) {
      int ky = 0;
      const int jj = mr_fold(y, I.ny, I.bcy, &ky) * I.nx;
      *z = (szero | (ky == 1 ? sfm : 0u)) | ((sneg ^ (ky == 2 ? syflip : 0u)) << 16);
#pragma unroll
      for (int q = 0; q < NQ; ++q) v[q] = U[soff[q] + jj];
    };
    auto store = [&](int y, const double* v, unsigned z) {
      double* d = mom[kx_slot(y, KX_MR)];
#pragma unroll
      for (int q = 0; q < NQ; ++q)
        if (tid + q * MR_BLOCK < NROW)
          d[tid + q * MR_BLOCK] = ((z >> q) & 1u) ? 0.0 : (((z >> (16 + q)) & 1u) ? -v[q] : v[q]);
    };
    /* ghosts of the stored rows y .. y+nr-1 that hold prescribed data,
       overwritten by the threads that stored them */
    auto prescribe = [&](int y, int nr) {
#pragma unroll 1
      for (int r = y; r < y + nr; ++r)
#pragma unroll 1
        for (int k = tid; k < NROW; k += MR_BLOCK) {
          const int pl = k / KX_XW;
          double v;
          if (mr_presc(I, pl / 3, pl % 3, xs + k % KX_XW, r, tb, &v) ||
              (GB == 2 && mr_step_val(I, U, pl / 3, pl % 3, xs + k % KX_XW, r, &v)))
            mom[kx_slot(r, KX_MR)][k] = v;
        }
    };
    /* prologue: moment rows y0-2 .. y0+3 */
#pragma unroll 1
    for (int y = tl.y0 - 2; y <= tl.y0 + 3; y += 2) {
      double a[NQ], b[NQ];
      unsigned za, zb;
      fetch(y, a, &za);
      fetch(y + 1, b, &zb);
      store(y, a, za);
      store(y + 1, b, zb);
    }
    if (GB && mr_presc_rows<GB == 2>(I, xs, KX_XW, tl.y0 - 2, 6)) prescribe(tl.y0 - 2, 6);
    __syncthreads();
    for (int s = 0; 4 * s <= tl.rows + 1; ++s) {
      const int r0 = tl.y0 - 1 + 4 * s;    /* rows r0 .. r0+3 are reconstructed */
      const int r = r0 + ry;
      if (r <= ylast) {
        double f[9];
        if constexpr (NK == 4) {
          /* characteristic-wise Step 1: x faces from the x set, y faces from the y set */
          f[8] = 0.0;
          kx_face_data_ch<BP, 0>(mom, kx_slot(r - 1, KX_MR), kx_slot(r, KX_MR), kx_slot(r + 1, KX_MR), cx + 1, I.W,
                                 I.gam, f, &f[8]);
          kx_face_data_ch<BP, 1>(mom, kx_slot(r - 1, KX_MR), kx_slot(r, KX_MR), kx_slot(r + 1, KX_MR), cx + 1, I.W,
                                 I.gam, f, &f[8]);
        } else {
          kx_face_data<NK, BP>(mom, kx_slot(r - 1, KX_MR), kx_slot(r, KX_MR), kx_slot(r + 1, KX_MR), cx + 1, I.W,
                               I.tc == 4 ? I.tvb_mh2 : -1.0, f);
        }
        const int sf = kx_slot(r, KX_FR);
#pragma unroll
        for (int k = 0; k < 9; ++k) fd[sf][k][cx] = f[k];
      }
      /* moment rows r0+5 .. r0+8 (up to ylast+1) for the next step: fetched
         now, stored (into the slots of rows r0-5 .. r0-2, which this step
         does not read) once the flags below are formed */
      double v[4][NQ];
      unsigned z[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) fetch(r0 + 5 + k, v[k], &z[k]);   /* rows past ylast+1: clamped, unused */
      __syncthreads();
      /* flags of row r0-1+ry from the face data of rows rf-1 .. rf+1 */
      const int rf = r0 - 1 + ry, x = xs + 1 + cx;
      if (rf >= tl.y0 && rf < tl.y0 + tl.rows && cx >= 1 && cx <= KX_W - 2 && x < I.nx + I.fhalo) {
#pragma clang fp contract(off)
        const int a = kx_slot(rf, KX_FR), b = kx_slot(rf - 1, KX_FR), u = kx_slot(rf + 1, KX_FR);
        if (I.tc == 4) {   /* TVB: the cell's own verdict */
          fl[(long long)(rf + I.fhalo) * I.fex + (x + I.fhalo)] = (unsigned char)(fd[a][0][cx] != 0.0);
        } else {
          double J = 0.0, len = 0.0;
          const double vl = 0.5 * (fd[a][4][cx] + fd[a][5][cx - 1]);
          if (vl > 0.0 && !(GB ? mr_wall_x<GB == 2>(I, x, rf, tb) : mr_wall(x, I.nx, I.bcx))) { J += I.dy * (fd[a][0][cx] - fd[a][1][cx - 1]); len += I.dy; }
          const double vr = 0.5 * (fd[a][5][cx] + fd[a][4][cx + 1]);
          if (-vr > 0.0 && !(GB ? mr_wall_x<GB == 2>(I, x + 1, rf, tb) : mr_wall(x + 1, I.nx, I.bcx))) { J += I.dy * (fd[a][1][cx] - fd[a][0][cx + 1]); len += I.dy; }
          const double vb = 0.5 * (fd[a][6][cx] + fd[b][7][cx]);
          if (vb > 0.0 && !(GB ? mr_wall_y<GB == 2>(I, x, rf, tb) : mr_wall(rf, I.ny, I.bcy))) { J += I.dx * (fd[a][2][cx] - fd[b][3][cx]); len += I.dx; }
          const double vt = 0.5 * (fd[a][7][cx] + fd[u][6][cx]);
          if (-vt > 0.0 && !(GB ? mr_wall_y<GB == 2>(I, x, rf + 1, tb) : mr_wall(rf + 1, I.ny, I.bcy))) { J += I.dx * (fd[a][3][cx] - fd[u][2][cx]); len += I.dx; }
          const double num = fabs(J);
          const double den = I.dx * I.dx * len * fd[a][8][cx];
          fl[(long long)(rf + I.fhalo) * I.fex + (x + I.fhalo)] = (unsigned char)(num > den);
          if (aleph && x >= 0 && x < I.nx && rf >= 0 && rf < I.ny) {
            const long long cell = (long long)rf * I.nx + x;
            aleph[2 * cell] = num;
            aleph[2 * cell + 1] = den;
          }
        }
      }
#pragma unroll
      for (int k = 0; k < 4; ++k)
        if (r0 + 5 + k <= ylast + 1) store(r0 + 5 + k, v[k], z[k]);
      if (GB && mr_presc_rows<GB == 2>(I, xs, KX_XW, r0 + 5, min(4, ylast - r0 - 3))) prescribe(r0 + 5, min(4, ylast - r0 - 3));
      __syncthreads();
    }
  }
}

/* gb: 0 no per-side boundary data in the list, 1 ghosts that hold a
   prescribed state, 2 also a step (NK = 3, 4) */
extern "C" hipError_t mr_launch_kxrcf2(hipStream_t s, int nk, int bp, int gb, mr_inst* d, const mr_tile2* t, int nt,
                                       int stage) {
  if (nt <= 0) return hipSuccess;
  const dim3 G(nt), B(MR_BLOCK);
#define MR_LK(NK_, BP_)                                                                                   \
  do {                                                                                                    \
    if (gb == 2 && NK_ > 1) hipLaunchKernelGGL((k2_kxrcf<NK_, BP_, 2>), G, B, 0, s, d, t, nt, stage);      \
    else if (gb) hipLaunchKernelGGL((k2_kxrcf<NK_, BP_, 1>), G, B, 0, s, d, t, nt, stage);                \
    else hipLaunchKernelGGL((k2_kxrcf<NK_, BP_, 0>), G, B, 0, s, d, t, nt, stage);                        \
  } while (0)
  if (nk == 1) { if (bp) MR_LK(1, true); else MR_LK(1, false); }
  else if (nk == 3) { if (bp) MR_LK(3, true); else MR_LK(3, false); }
  else if (nk == 4) { if (bp) MR_LK(4, true); else MR_LK(4, false); }   /* characteristic-wise */
  else return hipErrorInvalidValue;
#undef MR_LK
  return hipGetLastError();
}
