/* HIP kernels of the MR-HWENO operator for gfx950 (FP64 throughout).
 *
 * One SSP-RK3 step (eq. Runge-Kutta) is the launch sequence
 *   k_reduce(0)  -> k_finalize                      (dt from U^n, CFL)
 *   per stage s = 0, 1, 2:
 *     [k_reduce(s) for Lax-Friedrichs alpha when s > 0]
 *     k{1,2}_summary -> k{1,2}_flags                (Step 2.1, KXRCF)
 *     k{1,2}_stage(s)                               (Steps 1, 2.2, 2.3, fluxes,
 *                                                    residual, RK combination)
 * Every kernel takes a work list spanning all instances, so one launch
 * serves a whole batch of problems of different sizes.
 *
 * Modified first moments of troubled cells replace those of the stage input
 * (Step 2.2).  Within a stage they are computed from the unmodified input
 * (Jacobi); the RK combination uses the modified stage input, and the
 * modification of U^n made in the first stage is reapplied on the fly in
 * stages two and three from the stage-1 flags.
 */
#include "mr_device.h"

#define MR_BLOCK 256
/* occupancy target for the reconstruction kernels: the compiler schedules
   for at most 512 / MR_WAVES VGPRs per lane instead of the whole file */
#ifndef MR_WAVES
#define MR_WAVES 2
#endif
#define MR_OCC __attribute__((amdgpu_waves_per_eu(MR_WAVES)))

/* =================================================================== helpers */
struct mr_grid {
  const double* U;  /* state base: comp c, moment m plane at U + (c*nm + m)*P */
  long long P;
  int nx, ny, bcx, bcy, nm;
};

/* moment m of component c at cell (i, j) with ghost handling */
MR_INL double mr_ld(const mr_grid& g, int c, int m, int i, int j) {
  bool z = false;
  const int ii = mr_fold(i, g.nx, g.bcx, &z);
  const int jj = (g.nm == 3) ? mr_fold(j, g.ny, g.bcy, &z) : 0;
  if (z && m > 0) return 0.0;
  return g.U[(long long)(c * g.nm + m) * g.P + (long long)jj * g.nx + ii];
}

/* flag of cell (i, j) from an extended plane with halo h (clamped) */
MR_INL int mr_flag(const unsigned char* fl, int ex, int ey, int h, int i, int j) {
  int a = i + h, b = j + h;
  a = a < 0 ? 0 : (a >= ex ? ex - 1 : a);
  b = b < 0 ? 0 : (b >= ey ? ey - 1 : b);
  return fl[(long long)b * ex + a];
}

/* ----------------------------------------------------- 2D stencil + Step 1 */
/* Final Gauss-Lobatto values of component c of cell (x, y): Step 1 on the
 * stage input, or, for a troubled cell, Step 1 again with the first moments
 * of the troubled cells of its stencil replaced (Steps 2.2, 2.3).
 * ve/we receive the cell's own (possibly modified) first moments. */
/* Steps 2.2/2.3 input: first moments of the troubled cells of the stencil of
 * (x, y) replaced by their modified values (Jacobi, from the unmodified
 * stage input). */
MR_INL void mr2_modify_stencil(const mr_grid& g, int c, int x, int y, const int* fs,
                               double* v, double* w) {
#pragma unroll
  for (int l = 0; l < 9; ++l) {
    if (!fs[l]) continue;
    const int xs = x + l % 3 - 1, ys = y + l / 3 - 1;
    v[l] = mr_modified_moment(mr_ld(g, c, 0, xs - 1, ys), mr_ld(g, c, 0, xs + 1, ys),
                              mr_ld(g, c, 1, xs - 1, ys), mr_ld(g, c, 1, xs + 1, ys));
    w[l] = mr_modified_moment(mr_ld(g, c, 0, xs, ys - 1), mr_ld(g, c, 0, xs, ys + 1),
                              mr_ld(g, c, 2, xs, ys - 1), mr_ld(g, c, 2, xs, ys + 1));
  }
}

/* Final Gauss-Lobatto values of component c of cell (x, y): Step 1 on the
 * stage input, or, for a troubled cell, Step 1 again with the first moments
 * of the troubled cells of its stencil replaced (Steps 2.2, 2.3).
 * ue/ve/we receive the cell's own (possibly modified) moments. */
template <bool BP>
MR_INL void mr2_cell_values(const mr_grid& g, const mr_inst& I, const unsigned char* fl,
                            int c, int x, int y, double out[16], double* ue, double* ve, double* we) {
  double u[9], v[9], w[9];
  int fs[9];
#pragma unroll
  for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
    for (int dx = -1; dx <= 1; ++dx) {
      const int l = (dx + 1) + 3 * (dy + 1);
      u[l] = mr_ld(g, c, 0, x + dx, y + dy);
      v[l] = mr_ld(g, c, 1, x + dx, y + dy);
      w[l] = mr_ld(g, c, 2, x + dx, y + dy);
      fs[l] = mr_flag(fl, I.fex, I.fey, I.fhalo, x + dx, y + dy);
    }
  if (fs[4]) mr2_modify_stencil(g, c, x, y, fs, v, w);
  *ue = u[4];
  *ve = v[4];
  *we = w[4];
  mr_recon2d<BP>(u, v, w, I.W, out);
}

/* U^n with the stage-1 modification applied at cell (x, y), component c */
MR_INL void mr2_un_mod(const mr_grid& g, const unsigned char* fl1, const mr_inst& I,
                       int c, int x, int y, double* u, double* v, double* w) {
  *u = mr_ld(g, c, 0, x, y);
  if (mr_flag(fl1, I.fex, I.fey, I.fhalo, x, y)) {
    *v = mr_modified_moment(mr_ld(g, c, 0, x - 1, y), mr_ld(g, c, 0, x + 1, y),
                            mr_ld(g, c, 1, x - 1, y), mr_ld(g, c, 1, x + 1, y));
    *w = mr_modified_moment(mr_ld(g, c, 0, x, y - 1), mr_ld(g, c, 0, x, y + 1),
                            mr_ld(g, c, 2, x, y - 1), mr_ld(g, c, 2, x, y + 1));
  } else {
    *v = mr_ld(g, c, 1, x, y);
    *w = mr_ld(g, c, 2, x, y);
  }
}

template <int NC, int D>
MR_INL void mr_numflux(const double* a, const double* b, double gam, double alpha, double* f) {
  if (NC == 1) f[0] = mr_lf(a[0], b[0], alpha);
  else mr_hllc<NC, D>(a, b, gam, f);
}

template <int NC, int D>
MR_INL void mr_physflux(const double* u, double gam, double* f) {
  if (NC == 1) f[0] = 0.5 * u[0] * u[0];
  else mr_euler_flux<NC, D>(u, gam, f);
}

/* ================================================================ reduction */
/* Max wave speeds over the cell averages of the stage input (reading: dt
 * from U^n; Lax-Friedrichs alpha from every stage input), plus the
 * non-physical-state check.  One work item = up to MR_BLOCK cells. */
/* block-wide max of (ax, ay), result valid in thread 0 */
MR_INL void mr_block_max2(double* ax, double* ay, double* sh) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    *ax = fmax(*ax, __shfl_xor(*ax, o));
    *ay = fmax(*ay, __shfl_xor(*ay, o));
  }
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) { sh[2 * w] = *ax; sh[2 * w + 1] = *ay; }
  __syncthreads();
  if (threadIdx.x == 0)
    for (int k = 1; k < MR_BLOCK / 64; ++k) { *ax = fmax(*ax, sh[2 * k]); *ay = fmax(*ay, sh[2 * k + 1]); }
}

/* Each work group takes a contiguous run of `chunk` work items, keeps a
 * running max per instance and publishes it with one atomic per instance
 * run (max is exact, so the result does not depend on the order). */
__global__ __launch_bounds__(MR_BLOCK) void k_reduce(mr_inst* insts, const mr_tile1* tiles, int ntiles,
                                                     int stage, int chunk) {
#pragma clang fp contract(off)
  __shared__ double sh[2 * (MR_BLOCK / 64)];
  const int t0 = blockIdx.x * chunk, t1 = min(ntiles, t0 + chunk);
  int cur = -1;
  double ax = 0.0, ay = 0.0;
  int bad = 0;
  for (int t = t0; t <= t1; ++t) {
    const int inst = (t < t1) ? tiles[t].inst : -2;
    if (inst != cur && cur >= 0) {
      /* flush the finished instance (uniform across the block) */
      mr_inst& J = insts[cur];
      const int anybad = __syncthreads_or(bad);
      mr_block_max2(&ax, &ay, sh);
      if (threadIdx.x == 0) {
        if (stage == 0) {
          atomicMax(&J.amax[0], mr_dbits(ax));
          atomicMax(&J.amax[1], mr_dbits(ay));
          if (anybad) atomicOr(&J.err, 1);
        } else {
          atomicMax(&J.lfa[stage], mr_dbits(ax));
        }
      }
      ax = ay = 0.0;
      bad = 0;
    }
    cur = inst;
    if (t >= t1) break;
    const mr_tile1 tl = tiles[t];
    mr_inst& I = insts[tl.inst];
    const double* U;
    if (stage == 0) {
      if (I.err) continue;
      U = I.buf[I.cur];
    } else {
      if (!I.active || I.flux != 0) continue;
      U = I.p_out[stage - 1];
    }
    const int k = tl.start + (int)threadIdx.x;
    if (k < tl.start + tl.count) {
      const long long P = I.plane;
      const int nm = I.dim + 1;
      if (I.flux == 0) {
        const double a = fabs(U[k]);
        ax = fmax(ax, a);
        ay = fmax(ay, a);
        bad |= !(a <= 1.0e300);
      } else {
        double u[4];
        for (int c = 0; c < I.nc; ++c) u[c] = U[(long long)c * nm * P + k];
        double ke = u[1] * u[1];
        if (I.nc == 4) ke += u[2] * u[2];
        const double p = (I.gam - 1.0) * (u[I.nc - 1] - 0.5 * ke / u[0]);
        const double cs = sqrt(I.gam * p / u[0]);
        const double sx = fabs(u[1] / u[0]) + cs;
        const double sy = (I.nc == 4) ? fabs(u[2] / u[0]) + cs : 0.0;
        const int b = !(u[0] > 0.0) || !(p > 0.0) || !(sx <= 1.0e300) || !(sy <= 1.0e300);
        bad |= b;
        if (!b) { ax = fmax(ax, sx); ay = fmax(ay, sy); }
      }
    }
  }
}

/* Time step of the current step and the state rotation, one thread per
 * instance.  Reading for dt: cfl*dx/alpha (1D), cfl/(ax/dx + ay/dy) (2D),
 * clipped to the final time. */
__global__ void k_finalize(mr_inst* insts, int n, int probe) {
#pragma clang fp contract(off)
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  mr_inst& I = insts[q];
  const double ax = mr_bitsd(I.amax[0]), ay = mr_bitsd(I.amax[1]);
  if (probe) {
    /* one-off evaluation of L(U) or of the reconstruction: only the
       Lax-Friedrichs constant of the given state is needed */
    I.lfa[0] = mr_dbits(ax);
    I.amax[0] = 0ull;
    I.amax[1] = 0ull;
    return;
  }
  I.amax[0] = 0ull;
  I.amax[1] = 0ull;
  I.lfa[1] = 0ull;
  I.lfa[2] = 0ull;
  if (I.err) {
    if (!I.rolled) {
      /* keep the last good state: the previous U^n is still intact */
      if (I.steps > 0) {
        I.t = I.t_prev;
        I.steps -= 1;
        I.cur = (I.cur + 2) % 3;
      }
      I.rolled = 1;
    }
    I.active = 0;
    return;
  }
  double dt = (I.dim == 1) ? I.cfl * I.dx / ax : I.cfl / (ax / I.dx + ay / I.dy);
  const double rem = I.t_final - I.t;
  bool last = false;
  if (dt >= rem) { dt = rem; last = true; }
  if (!(dt > 0.0)) { I.active = 0; return; }
  I.active = 1;
  I.dt = dt;
  I.t_prev = I.t;
  I.t = last ? I.t_final : I.t + dt;
  I.steps += 1;
  I.lfa[0] = mr_dbits(ax);
  const int c = I.cur;
  double* b0 = I.buf[c];
  double* b1 = I.buf[(c + 1) % 3];
  double* b2 = I.buf[(c + 2) % 3];
  I.p_un = b0;
  I.p_in[0] = b0; I.p_out[0] = b1;
  I.p_in[1] = b1; I.p_out[1] = b2;
  I.p_in[2] = b2; I.p_out[2] = b1;
  I.cur = (c + 1) % 3;
}

/* ================================================================ 1D passes */
/* KXRCF face data per cell over the extended range [-3, nx+3):
 * plane 0: own value at x_{i-1/2}, 1: at x_{i+1/2}, 2: velocity at
 * x_{i-1/2}, 3: velocity at x_{i+1/2}, 4: max |u| over the 4 GL points. */
template <bool BP>
__global__ __launch_bounds__(MR_BLOCK) MR_OCC void k1_summary(mr_inst* insts, const mr_tile1* tiles, int ntiles, int stage) {
  for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const mr_tile1 tl = tiles[t];
    const mr_inst& I = insts[tl.inst];
    if (stage < 3 && !I.active) continue;
    if (I.tc != 1 && I.tc != 3) continue;
    const int e = tl.start + (int)threadIdx.x;
    if (e >= tl.start + tl.count) continue;
    const int i = e - I.shalo;
    mr_grid g{stage < 3 ? I.p_in[stage] : I.buf[0], I.plane, I.nx, 1, I.bcx, I.bcy, 2};
    double r[4];
    mr_recon1d<BP>(mr_ld(g, 0, 0, i - 1, 0), mr_ld(g, 0, 0, i, 0), mr_ld(g, 0, 0, i + 1, 0),
                   mr_ld(g, 0, 1, i - 1, 0), mr_ld(g, 0, 1, i, 0), mr_ld(g, 0, 1, i + 1, 0), I.W, r);
    double vl = r[0], vr = r[3];
    if (I.flux == 1) {
      double m[4];
      mr_recon1d<BP>(mr_ld(g, 1, 0, i - 1, 0), mr_ld(g, 1, 0, i, 0), mr_ld(g, 1, 0, i + 1, 0),
                     mr_ld(g, 1, 1, i - 1, 0), mr_ld(g, 1, 1, i, 0), mr_ld(g, 1, 1, i + 1, 0), I.W, m);
      vl = m[0] / r[0];
      vr = m[3] / r[3];
    }
    double nrm = 0.0;
#pragma unroll
    for (int k = 0; k < 4; ++k) nrm = fmax(nrm, fabs(r[k]));
    const long long SE = I.sex;
    I.summ[0 * SE + e] = r[0];
    I.summ[1 * SE + e] = r[3];
    I.summ[2 * SE + e] = vl;
    I.summ[3 * SE + e] = vr;
    I.summ[4 * SE + e] = nrm;
  }
}

/* Troubled-cell flags, eq. (KXRCF) with eq. (line-integral-average), over
 * [-2, nx+2); tc = 0 / 2 write all-zero / all-one maps. */
__global__ __launch_bounds__(MR_BLOCK) void k1_flags(mr_inst* insts, const mr_tile1* tiles, int ntiles, int stage) {
#pragma clang fp contract(off)
  for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const mr_tile1 tl = tiles[t];
    mr_inst& I = insts[tl.inst];
    if (stage < 3 && !I.active) continue;
    const int e = tl.start + (int)threadIdx.x;
    if (e >= tl.start + tl.count) continue;
    unsigned char* fl = I.flags[(stage == 0 || stage == 3) ? 0 : 1];
    if (I.tc == 0 || I.tc == 2) { fl[e] = (unsigned char)(I.tc == 2); continue; }
    const int s = e + (I.shalo - I.fhalo);   /* same cell in the summary plane */
    const long long SE = I.sex;
    const double* S = I.summ;
    const double jl = S[0 * SE + s] - S[1 * SE + s - 1];
    const double vl = 0.5 * (S[2 * SE + s] + S[3 * SE + s - 1]);
    const double jr = S[1 * SE + s] - S[0 * SE + s + 1];
    const double vr = 0.5 * (S[3 * SE + s] + S[2 * SE + s + 1]);
    const double J = jl * (vl > 0.0 ? 1.0 : 0.0) + jr * (-vr > 0.0 ? 1.0 : 0.0);
    const double num = fabs(J);
    const double den = I.dx * I.dx * S[4 * SE + s];
    fl[e] = (unsigned char)(num > den);
    if (I.aleph) {
      const int i = e - I.fhalo;
      if (i >= 0 && i < I.nx) { I.aleph[2 * i] = num; I.aleph[2 * i + 1] = den; }
    }
  }
}

/* 1D stage: one thread per cell of a block-sized tile; the two edge threads
 * are ring cells that only supply face values.  mode 0..2 = RK stage,
 * mode 3 = write L(U) (input p_in[0], output p_out[0]). */
template <int NC, bool BP>
__global__ __launch_bounds__(MR_BLOCK) MR_OCC void k1_stage(mr_inst* insts, const mr_tile1* tiles, int ntiles, int mode) {
  __shared__ double s_tr[MR_BLOCK * NC];
  __shared__ double s_fl[MR_BLOCK * NC];
  const int cs = threadIdx.x;
  for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const mr_tile1 tl = tiles[t];
    const mr_inst& I = insts[tl.inst];
    if (mode < 3 && !I.active) continue;
    const int st = mode == 3 ? 0 : mode;
    const mr_grid g{I.p_in[st], I.plane, I.nx, 1, I.bcx, I.bcy, 2};
    const unsigned char* fl = I.flags[(mode == 0 || mode == 3) ? 0 : 1];
    const int x = tl.start - 1 + cs;
    const int fh = I.fhalo;
    const int f0 = mr_flag(fl, I.fex, 1, fh, x, 0);
    int fm = 0, fp = 0;
    if (f0) { fm = mr_flag(fl, I.fex, 1, fh, x - 1, 0); fp = mr_flag(fl, I.fex, 1, fh, x + 1, 0); }
    double val[NC][4], vt[NC][2];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const double um = mr_ld(g, c, 0, x - 1, 0), u0 = mr_ld(g, c, 0, x, 0), up = mr_ld(g, c, 0, x + 1, 0);
      double vm = mr_ld(g, c, 1, x - 1, 0), v0 = mr_ld(g, c, 1, x, 0), vp = mr_ld(g, c, 1, x + 1, 0);
      if (f0) {
        /* Steps 2.2/2.3: Step 1 again with the troubled cells' first moments modified */
        if (fm) vm = mr_modified_moment(mr_ld(g, c, 0, x - 2, 0), u0, mr_ld(g, c, 1, x - 2, 0), v0);
        vp = fp ? mr_modified_moment(u0, mr_ld(g, c, 0, x + 2, 0), v0, mr_ld(g, c, 1, x + 2, 0)) : vp;
        v0 = mr_modified_moment(um, up, mr_ld(g, c, 1, x - 1, 0), mr_ld(g, c, 1, x + 1, 0));
      }
      vt[c][0] = u0;
      vt[c][1] = v0;
      mr_recon1d<BP>(um, u0, up, vm, v0, vp, I.W, val[c]);
      s_tr[cs * NC + c] = val[c][3];
    }
    __syncthreads();
    const double alpha = (NC == 1) ? mr_bitsd(I.lfa[st]) : 0.0;
    double fh_[NC];
    if (cs >= 1) {
      double a[NC], b[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) { a[c] = s_tr[(cs - 1) * NC + c]; b[c] = val[c][0]; }
      mr_numflux<NC, 0>(a, b, I.gam, alpha, fh_);
#pragma unroll
      for (int c = 0; c < NC; ++c) s_fl[cs * NC + c] = fh_[c];
    }
    __syncthreads();
    const bool out = cs >= 1 && cs <= MR_BLOCK - 2 && x < I.nx && x < tl.start + tl.count;
    if (out) {
      double F[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) F[c] = 0.0;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        double pt[NC], f[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) pt[c] = val[c][q];
        mr_physflux<NC, 0>(pt, I.gam, f);
#pragma unroll
        for (int c = 0; c < NC; ++c) F[c] += glw(q) * f[c];
      }
      double* O = I.p_out[st];
      const long long P = I.plane;
      const double dt = I.dt;
      const mr_grid gn{I.p_un, I.plane, I.nx, 1, I.bcx, I.bcy, 2};
      const int f1 = (mode == 1 || mode == 2) ? mr_flag(I.flags[0], I.fex, 1, fh, x, 0) : 0;
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        const double fm_ = s_fl[cs * NC + c], fp_ = s_fl[(cs + 1) * NC + c];
        const double L0 = -(fp_ - fm_) / I.dx;
        const double L1 = -(fp_ + fm_) / (2.0 * I.dx) + F[c] / I.dx;
        double r0, r1;
        if (mode == 3) { r0 = L0; r1 = L1; }
        else if (mode == 0) { r0 = vt[c][0] + dt * L0; r1 = vt[c][1] + dt * L1; }
        else {
          const double a = mode == 1 ? 0.75 : 1.0 / 3.0, b = mode == 1 ? 0.25 : 2.0 / 3.0;
          const double un0 = mr_ld(gn, c, 0, x, 0);
          const double un1 = f1 ? mr_modified_moment(mr_ld(gn, c, 0, x - 1, 0), mr_ld(gn, c, 0, x + 1, 0),
                                                      mr_ld(gn, c, 1, x - 1, 0), mr_ld(gn, c, 1, x + 1, 0))
                                : mr_ld(gn, c, 1, x, 0);
          r0 = a * un0 + b * vt[c][0] + b * dt * L0;
          r1 = a * un1 + b * vt[c][1] + b * dt * L1;
        }
        O[(long long)(c * 2 + 0) * P + x] = r0;
        O[(long long)(c * 2 + 1) * P + x] = r1;
      }
    }
    __syncthreads();
  }
}

/* 1D final Gauss-Lobatto values of interior cells: gl[(c*4 + k)*nx + i]. */
template <int NC, bool BP>
__global__ __launch_bounds__(MR_BLOCK) MR_OCC void k1_values(mr_inst* insts, const mr_tile1* tiles, int ntiles, double* gl) {
  for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const mr_tile1 tl = tiles[t];
    const mr_inst& I = insts[tl.inst];
    const int x = tl.start + (int)threadIdx.x;
    if (x >= tl.start + tl.count) continue;
    const mr_grid g{I.p_in[0], I.plane, I.nx, 1, I.bcx, I.bcy, 2};
    const unsigned char* fl = I.flags[0];
    const int fh = I.fhalo;
    const int f0 = mr_flag(fl, I.fex, 1, fh, x, 0);
    const int fm = mr_flag(fl, I.fex, 1, fh, x - 1, 0), fp = mr_flag(fl, I.fex, 1, fh, x + 1, 0);
    for (int c = 0; c < NC; ++c) {
      const double um = mr_ld(g, c, 0, x - 1, 0), u0 = mr_ld(g, c, 0, x, 0), up = mr_ld(g, c, 0, x + 1, 0);
      double vm = mr_ld(g, c, 1, x - 1, 0), v0 = mr_ld(g, c, 1, x, 0), vp = mr_ld(g, c, 1, x + 1, 0);
      if (f0) {
        if (fm) vm = mr_modified_moment(mr_ld(g, c, 0, x - 2, 0), u0, mr_ld(g, c, 1, x - 2, 0), v0);
        if (fp) vp = mr_modified_moment(u0, mr_ld(g, c, 0, x + 2, 0), v0, mr_ld(g, c, 1, x + 2, 0));
        v0 = mr_modified_moment(um, up, mr_ld(g, c, 1, x - 1, 0), mr_ld(g, c, 1, x + 1, 0));
      }
      double r[4];
      mr_recon1d<BP>(um, u0, up, vm, v0, vp, I.W, r);
      for (int k = 0; k < 4; ++k) gl[(long long)(c * 4 + k) * I.plane + x] = r[k];
    }
  }
}

/* ================================================================ 2D passes */
/* KXRCF face data per cell over the extended range [-3, n+3)^2, planes:
 * 0..3 Gauss-Lobatto-weighted mean of the indicator variable on the left,
 * right, bottom, top face; 4..7 the same for the normal velocity; 8 max |u|
 * over the 16 points. */
template <bool BP>
__global__ __launch_bounds__(MR_BLOCK) MR_OCC void k2_summary(mr_inst* insts, const mr_tile1* tiles, int ntiles, int stage) {
  for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const mr_tile1 tl = tiles[t];
    const mr_inst& I = insts[tl.inst];
    if (stage < 3 && !I.active) continue;
    if (I.tc != 1 && I.tc != 3) continue;
    const int e = tl.start + (int)threadIdx.x;
    if (e >= tl.start + tl.count) continue;
    const int i = e % I.sex - I.shalo, j = e / I.sex - I.shalo;
    const mr_grid g{stage < 3 ? I.p_in[stage] : I.buf[0], I.plane, I.nx, I.ny, I.bcx, I.bcy, 3};
    const mr_wconst W = I.W;
    /* component 0 gives the indicator variable; for Euler, components 1
       and 2 give the velocities on the x and y faces */
    double rho[16];
    double sl = 0.0, sr = 0.0, sb = 0.0, st = 0.0, nrm = 0.0;
    double vl = 0.0, vr = 0.0, vb = 0.0, vt = 0.0;
    const int ncomp = I.flux == 1 ? 3 : 1;
#pragma unroll 1
    for (int c = 0; c < ncomp; ++c) {
      double u[9], v[9], w[9], r[16];
#pragma unroll
      for (int l = 0; l < 9; ++l) {
        const int dx = l % 3 - 1, dy = l / 3 - 1;
        u[l] = mr_ld(g, c, 0, i + dx, j + dy);
        v[l] = mr_ld(g, c, 1, i + dx, j + dy);
        w[l] = mr_ld(g, c, 2, i + dx, j + dy);
      }
      mr_recon2d<BP>(u, v, w, W, r);
      if (c == 0) {
#pragma unroll
        for (int m = 0; m < 4; ++m) {
          sl += glw(m) * r[0 + 4 * m];
          sr += glw(m) * r[3 + 4 * m];
          sb += glw(m) * r[m];
          st += glw(m) * r[12 + m];
        }
#pragma unroll
        for (int k = 0; k < 16; ++k) { nrm = fmax(nrm, fabs(r[k])); rho[k] = r[k]; }
        vl = sl; vr = sr; vb = sb; vt = st;   /* Burgers: f'(u) = u */
        if (ncomp > 1) { vl = vr = vb = vt = 0.0; }
      } else if (c == 1) {
#pragma unroll
        for (int m = 0; m < 4; ++m) {
          vl += glw(m) * (r[0 + 4 * m] / rho[0 + 4 * m]);
          vr += glw(m) * (r[3 + 4 * m] / rho[3 + 4 * m]);
        }
      } else {
#pragma unroll
        for (int m = 0; m < 4; ++m) {
          vb += glw(m) * (r[m] / rho[m]);
          vt += glw(m) * (r[12 + m] / rho[12 + m]);
        }
      }
    }
    const long long SE = (long long)I.sex * I.sey;
    double* S = I.summ;
    S[0 * SE + e] = sl; S[1 * SE + e] = sr; S[2 * SE + e] = sb; S[3 * SE + e] = st;
    S[4 * SE + e] = vl; S[5 * SE + e] = vr; S[6 * SE + e] = vb; S[7 * SE + e] = vt;
    S[8 * SE + e] = nrm;
  }
}

/* Troubled-cell flags, eq. (KXRCF_) with eq. (line-integral-average_), over
 * [-2, n+2)^2, evaluated as |J| > h^2 |dI^-| ||u|| with h = dx. */
__global__ __launch_bounds__(MR_BLOCK) void k2_flags(mr_inst* insts, const mr_tile1* tiles, int ntiles, int stage) {
#pragma clang fp contract(off)
  for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const mr_tile1 tl = tiles[t];
    mr_inst& I = insts[tl.inst];
    if (stage < 3 && !I.active) continue;
    const int e = tl.start + (int)threadIdx.x;
    if (e >= tl.start + tl.count) continue;
    unsigned char* fl = I.flags[(stage == 0 || stage == 3) ? 0 : 1];
    if (I.tc == 0 || I.tc == 2) { fl[e] = (unsigned char)(I.tc == 2); continue; }
    const int i = e % I.fex - I.fhalo, j = e / I.fex - I.fhalo;
    const int sx = I.sex, d = I.shalo;
    const long long SE = (long long)sx * I.sey;
    const double* S = I.summ;
    const long long o = (long long)(j + d) * sx + (i + d);
    double J = 0.0, len = 0.0;
    const double vl = 0.5 * (S[4 * SE + o] + S[5 * SE + o - 1]);
    if (vl > 0.0) { J += I.dy * (S[0 * SE + o] - S[1 * SE + o - 1]); len += I.dy; }
    const double vr = 0.5 * (S[5 * SE + o] + S[4 * SE + o + 1]);
    if (-vr > 0.0) { J += I.dy * (S[1 * SE + o] - S[0 * SE + o + 1]); len += I.dy; }
    const double vb = 0.5 * (S[6 * SE + o] + S[7 * SE + o - sx]);
    if (vb > 0.0) { J += I.dx * (S[2 * SE + o] - S[3 * SE + o - sx]); len += I.dx; }
    const double vt = 0.5 * (S[7 * SE + o] + S[6 * SE + o + sx]);
    if (-vt > 0.0) { J += I.dx * (S[3 * SE + o] - S[2 * SE + o + sx]); len += I.dx; }
    const double num = fabs(J);
    const double den = I.dx * I.dx * len * S[8 * SE + o];
    fl[e] = (unsigned char)(num > den);
    if (I.aleph && i >= 0 && i < I.nx && j >= 0 && j < I.ny) {
      const long long cell = (long long)j * I.nx + i;
      I.aleph[2 * cell] = num;
      I.aleph[2 * cell + 1] = den;
    }
  }
}

/* reduce-scatter over the NC lanes of a cell: lane k receives sum_r a_r[k] */
template <int NC>
MR_INL double mr_rs(const double (&a)[NC], int k) {
  if (NC == 1) return a[0];
  const bool hi = (k & 2) != 0;
  const double s0 = hi ? a[0] : a[2], s1 = hi ? a[1] : a[3];
  const double k0 = hi ? a[2] : a[0], k1 = hi ? a[3] : a[1];
  const double b0 = k0 + __shfl_xor(s0, 2);
  const double b1 = k1 + __shfl_xor(s1, 2);
  const bool odd = (k & 1) != 0;
  const double s = odd ? b0 : b1, kk = odd ? b1 : b0;
  return kk + __shfl_xor(s, 1);
}

/* 2D stage kernel.  A work group owns a strip of CW = 256/NC consecutive
 * cells in x (two of them ring cells) and sweeps it upward over `rows` rows
 * plus one ring row below and one above.
 *
 * Moments: the rows y-2..y+2 of the strip (plus two columns each side) sit
 * in an LDS ring of five rows; each value is loaded from HBM once per work
 * group, with the boundary condition applied when it is loaded, and the
 * row needed next is fetched into registers while the current row is
 * computed.  Flags of rows y-1..y+1 sit in a three-row LDS ring.
 *
 * With NC = 4 the four lanes of a cell each reconstruct one conserved
 * component, then each lane takes one row eta_r of the cell's 4x4
 * Gauss-Lobatto grid for the volume integrals, the left-face flux at eta_r
 * and the bottom-face flux at xi_r.  The top-face flux of a row is the
 * bottom-face flux of the next one, so the residual of row j is completed
 * while row j+1 is processed.  mode 0..2 = RK stage, 3 = write L(U). */
template <int NC>
struct mr2_lds {
  static constexpr int CW = MR_BLOCK / NC;   /* strip cells incl. ring */
  static constexpr int XW = CW + 4;          /* staged columns */
  static constexpr int NP = 3 * NC;          /* staged planes */
  double mom[5][NP][XW];
  unsigned char flg[3][XW];
  double val[CW * NC * 16];
  double top[CW * NC * 4];
  double fs[CW * NC * 2];
};

/* one staged element: plane q (= 3 c + m) of row y, column col of the strip */
MR_INL double mr2_stage_ld(const mr_grid& g, int q, int x, int y) {
  return mr_ld(g, q / 3, q % 3, x, y);
}

template <int NC, bool BP>
__global__ __launch_bounds__(MR_BLOCK) MR_OCC void k2_stage(mr_inst* insts, const mr_tile2* tiles, int ntiles, int mode) {
  using S = mr2_lds<NC>;
  constexpr int CW = S::CW, XW = S::XW, NP = S::NP;
  constexpr int NE = (NP * XW + MR_BLOCK - 1) / MR_BLOCK;   /* staged values per thread per row */
  __shared__ S sh;
  const int tid = threadIdx.x;
  const int cs = tid / NC, k = tid % NC;
  const int comp = (NC == 1) ? 0 : k;
  for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const mr_tile2 tl = tiles[t];
    const mr_inst& I = insts[tl.inst];
    if (mode < 3 && !I.active) continue;
    const int st = mode == 3 ? 0 : mode;
    const mr_grid g{I.p_in[st], I.plane, I.nx, I.ny, I.bcx, I.bcy, 3};
    const mr_grid gn{I.p_un, I.plane, I.nx, I.ny, I.bcx, I.bcy, 3};
    const unsigned char* fl = I.flags[(mode == 0 || mode == 3) ? 0 : 1];
    const double rdx = I.rdx, rdy = I.rdy, dt = I.dt, gam = I.gam;
    const double alpha = (NC == 1) ? mr_bitsd(I.lfa[st]) : 0.0;
    double* O = I.p_out[st];
    const long long P = I.plane;
    const int xs0 = tl.x0 - 3;                 /* strip column 0 */
    const int x = tl.x0 - 1 + cs;
    const bool outx = cs >= 1 && cs <= CW - 2 && x < I.nx;
    /* ---- prologue: moment rows y0-3 .. y0+1, flag rows y0-2 .. y0 ---- */
    for (int r = tl.y0 - 3; r <= tl.y0 + 1; ++r) {
      const int sl = ((r % 5) + 5) % 5;
      for (int e = tid; e < NP * XW; e += MR_BLOCK)
        sh.mom[sl][e / XW][e % XW] = mr2_stage_ld(g, e / XW, xs0 + e % XW, r);
    }
    for (int r = tl.y0 - 2; r <= tl.y0; ++r) {
      const int sl = ((r % 3) + 3) % 3;
      for (int e = tid; e < XW; e += MR_BLOCK)
        sh.flg[sl][e] = (unsigned char)mr_flag(fl, I.fex, I.fey, I.fhalo, xs0 + e, r);
    }
    __syncthreads();
    double pAu = 0.0, pAv = 0.0, pAw = 0.0, pB0 = 0.0, pB1 = 0.0, pU = 0.0, pV = 0.0, pW = 0.0;
    for (int jr = -1; jr <= tl.rows; ++jr) {
      const int y = tl.y0 + jr;
      /* prefetch moment row y+3 and flag row y+2 (stored after this row) */
      double pre[NE];
      unsigned char pref = 0;
#pragma unroll
      for (int q = 0; q < NE; ++q) {
        const int e = tid + q * MR_BLOCK;
        pre[q] = (e < NP * XW) ? mr2_stage_ld(g, e / XW, xs0 + e % XW, y + 3) : 0.0;
      }
      if (tid < XW) pref = (unsigned char)mr_flag(fl, I.fex, I.fey, I.fhalo, xs0 + tid, y + 2);
      /* ---- Steps 1, 2.2, 2.3 for component `comp` of cell (x, y) ---- */
      double cu, cv, cw;
      {
        const int rm = ((y - 1) % 5 + 5) % 5, r0 = ((y % 5) + 5) % 5, rp = ((y + 1) % 5 + 5) % 5;
        const int fm = ((y - 1) % 3 + 3) % 3, f0 = ((y % 3) + 3) % 3, fp = ((y + 1) % 3 + 3) % 3;
        const int c0 = cs + 2;                    /* staged column of cell x */
        const int rr[3] = {rm, r0, rp}, ff[3] = {fm, f0, fp};
        double u[9], v[9], w[9];
        int fs[9];
#pragma unroll
        for (int dy = 0; dy < 3; ++dy)
#pragma unroll
          for (int dx = 0; dx < 3; ++dx) {
            const int l = dx + 3 * dy;
            u[l] = sh.mom[rr[dy]][3 * comp + 0][c0 + dx - 1];
            v[l] = sh.mom[rr[dy]][3 * comp + 1][c0 + dx - 1];
            w[l] = sh.mom[rr[dy]][3 * comp + 2][c0 + dx - 1];
            fs[l] = sh.flg[ff[dy]][c0 + dx - 1];
          }
        if (fs[4]) {
          /* troubled cell: first moments of the troubled cells of the
             stencil modified from the unmodified input (Jacobi) */
          const int r2m = ((y - 2) % 5 + 5) % 5, r2p = ((y + 2) % 5 + 5) % 5;
          const int rrr[5] = {r2m, rm, r0, rp, r2p};
#pragma unroll
          for (int dy = 0; dy < 3; ++dy)
#pragma unroll
            for (int dx = 0; dx < 3; ++dx) {
              const int l = dx + 3 * dy;
              if (!fs[l]) continue;
              const int cc = c0 + dx - 1;
              const int rw = rrr[dy + 1];
              v[l] = mr_modified_moment(sh.mom[rw][3 * comp][cc - 1], sh.mom[rw][3 * comp][cc + 1],
                                        sh.mom[rw][3 * comp + 1][cc - 1], sh.mom[rw][3 * comp + 1][cc + 1]);
              w[l] = mr_modified_moment(sh.mom[rrr[dy]][3 * comp][cc], sh.mom[rrr[dy + 2]][3 * comp][cc],
                                        sh.mom[rrr[dy]][3 * comp + 2][cc], sh.mom[rrr[dy + 2]][3 * comp + 2][cc]);
            }
        }
        cu = u[4];
        cv = v[4];
        cw = w[4];
        double val[16];
        mr_recon2d<BP>(u, v, w, I.W, val);
#pragma unroll
        for (int q = 0; q < 16; ++q) sh.val[(cs * NC + comp) * 16 + q] = val[q];
      }
      __syncthreads();
      /* ---- volume integrals and the fluxes this lane owns ---- */
      double F[NC], G[NC], XL0[NC], XL1[NC], YB0[NC], YB1[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) F[c] = G[c] = XL0[c] = XL1[c] = YB0[c] = YB1[c] = 0.0;
      const bool body = jr >= 0 && jr < tl.rows;
#pragma unroll
      for (int rr = 0; rr < 4 / NC; ++rr) {
        const int r = (NC == 1) ? rr : k;
        const double wr = glw(r), er = gln(r);
        if (body) {
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            double pt[NC], f[NC], gg[NC];
#pragma unroll
            for (int c = 0; c < NC; ++c) pt[c] = sh.val[(cs * NC + c) * 16 + q + 4 * r];
            if (NC == 4) mr_euler_fg(pt, gam, f, gg);
            else { f[0] = 0.5 * pt[0] * pt[0]; gg[0] = f[0]; }
            const double wq = glw(q) * wr;
#pragma unroll
            for (int c = 0; c < NC; ++c) { F[c] += wq * f[c]; G[c] += wq * gg[c]; }
          }
          if (cs >= 1) {
            double a[NC], b[NC], fh[NC];
#pragma unroll
            for (int c = 0; c < NC; ++c) {
              a[c] = sh.val[((cs - 1) * NC + c) * 16 + 3 + 4 * r];
              b[c] = sh.val[(cs * NC + c) * 16 + 4 * r];
            }
            mr_numflux<NC, 0>(a, b, gam, alpha, fh);
#pragma unroll
            for (int c = 0; c < NC; ++c) { XL0[c] += wr * fh[c]; XL1[c] += wr * er * fh[c]; }
          }
        }
        if (jr >= 0) {
          double a[NC], b[NC], gh[NC];
#pragma unroll
          for (int c = 0; c < NC; ++c) {
            a[c] = sh.top[(cs * NC + c) * 4 + r];
            b[c] = sh.val[(cs * NC + c) * 16 + r];
          }
          mr_numflux<NC, 1>(a, b, gam, alpha, gh);
#pragma unroll
          for (int c = 0; c < NC; ++c) { YB0[c] += wr * gh[c]; YB1[c] += wr * er * gh[c]; }
        }
      }
      /* lane k collects component k's sums */
      const double fF = mr_rs<NC>(F, k), fG = mr_rs<NC>(G, k);
      const double xl0 = mr_rs<NC>(XL0, k), xl1 = mr_rs<NC>(XL1, k);
      const double yb0 = mr_rs<NC>(YB0, k), yb1 = mr_rs<NC>(YB1, k);
      sh.fs[(cs * NC + comp) * 2 + 0] = xl0;
      sh.fs[(cs * NC + comp) * 2 + 1] = xl1;
      __syncthreads();
      /* the row below has consumed its top trace; store this row's */
#pragma unroll
      for (int q = 0; q < 4; ++q)
        sh.top[(cs * NC + comp) * 4 + q] = sh.val[(cs * NC + comp) * 16 + 12 + q];
      /* ring slots of rows y-2 (moments) and y-1 (flags) are free now */
      {
        const int sl = ((y + 3) % 5 + 5) % 5;
#pragma unroll
        for (int q = 0; q < NE; ++q) {
          const int e = tid + q * MR_BLOCK;
          if (e < NP * XW) sh.mom[sl][e / XW][e % XW] = pre[q];
        }
        if (tid < XW) sh.flg[((y + 2) % 3 + 3) % 3][tid] = pref;
      }
      /* ---- finish the row below: its top face is this row's bottom face ---- */
      if (jr >= 1 && outx) {
        const int yp = y - 1;
        const double Lu = pAu - (yb0 - pB0) * rdy;
        const double Lv = pAv - (yb1 - pB1) * rdy;
        const double Lw = pAw - (yb0 + pB0) * (0.5 * rdy);
        double r0, r1, r2;
        if (mode == 3) { r0 = Lu; r1 = Lv; r2 = Lw; }
        else if (mode == 0) { r0 = pU + dt * Lu; r1 = pV + dt * Lv; r2 = pW + dt * Lw; }
        else {
          const double a = mode == 1 ? 0.75 : 1.0 / 3.0, b = mode == 1 ? 0.25 : 2.0 / 3.0;
          double un, vn, wn;
          mr2_un_mod(gn, I.flags[0], I, comp, x, yp, &un, &vn, &wn);
          r0 = a * un + b * pU + b * dt * Lu;
          r1 = a * vn + b * pV + b * dt * Lv;
          r2 = a * wn + b * pW + b * dt * Lw;
        }
        const long long cell = (long long)yp * I.nx + x;
        O[(long long)(comp * 3 + 0) * P + cell] = r0;
        O[(long long)(comp * 3 + 1) * P + cell] = r1;
        O[(long long)(comp * 3 + 2) * P + cell] = r2;
      }
      /* ---- this row's partial residual (all but the top face) ---- */
      if (cs + 1 < CW) {
        const double xr0 = sh.fs[((cs + 1) * NC + comp) * 2 + 0];
        const double xr1 = sh.fs[((cs + 1) * NC + comp) * 2 + 1];
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
}

/* 2D final Gauss-Lobatto values of interior cells: gl[(c*16 + p)*plane + cell]. */
template <int NC, bool BP>
__global__ __launch_bounds__(MR_BLOCK) MR_OCC void k2_values(mr_inst* insts, const mr_tile1* tiles, int ntiles, double* gl) {
  for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const mr_tile1 tl = tiles[t];
    const mr_inst& I = insts[tl.inst];
    const int e = tl.start + (int)threadIdx.x;
    if (e >= tl.start + tl.count) continue;
    const int x = e % I.nx, y = e / I.nx;
    const mr_grid g{I.p_in[0], I.plane, I.nx, I.ny, I.bcx, I.bcy, 3};
    for (int c = 0; c < NC; ++c) {
      double val[16], a, b, d;
      mr2_cell_values<BP>(g, I, I.flags[0], c, x, y, val, &a, &b, &d);
      for (int p = 0; p < 16; ++p) gl[(long long)(c * 16 + p) * I.plane + e] = val[p];
    }
  }
}

/* ============================================================ host launchers */
extern "C" {

hipError_t mr_launch_reduce(hipStream_t s, mr_inst* d, const mr_tile1* t, int nt, int stage) {
  if (nt <= 0) return hipSuccess;
  const int chunk = nt > 2048 ? (nt + 2047) / 2048 : 1;
  const int grid = (nt + chunk - 1) / chunk;
  hipLaunchKernelGGL(k_reduce, dim3(grid), dim3(MR_BLOCK), 0, s, d, t, nt, stage, chunk);
  return hipGetLastError();
}

hipError_t mr_launch_finalize(hipStream_t s, mr_inst* d, int n, int probe) {
  hipLaunchKernelGGL(k_finalize, dim3((n + 63) / 64), dim3(64), 0, s, d, n, probe);
  return hipGetLastError();
}

hipError_t mr_launch_summary(hipStream_t s, int dim, int bp, mr_inst* d, const mr_tile1* t, int nt, int stage) {
  if (nt <= 0) return hipSuccess;
  if (dim == 1) {
    if (bp) hipLaunchKernelGGL(k1_summary<true>, dim3(nt), dim3(MR_BLOCK), 0, s, d, t, nt, stage);
    else hipLaunchKernelGGL(k1_summary<false>, dim3(nt), dim3(MR_BLOCK), 0, s, d, t, nt, stage);
  } else {
    if (bp) hipLaunchKernelGGL(k2_summary<true>, dim3(nt), dim3(MR_BLOCK), 0, s, d, t, nt, stage);
    else hipLaunchKernelGGL(k2_summary<false>, dim3(nt), dim3(MR_BLOCK), 0, s, d, t, nt, stage);
  }
  return hipGetLastError();
}

hipError_t mr_launch_flags(hipStream_t s, int dim, mr_inst* d, const mr_tile1* t, int nt, int stage) {
  if (nt <= 0) return hipSuccess;
  if (dim == 1) hipLaunchKernelGGL(k1_flags, dim3(nt), dim3(MR_BLOCK), 0, s, d, t, nt, stage);
  else hipLaunchKernelGGL(k2_flags, dim3(nt), dim3(MR_BLOCK), 0, s, d, t, nt, stage);
  return hipGetLastError();
}

hipError_t mr_launch_stage1(hipStream_t s, int nc, int bp, mr_inst* d, const mr_tile1* t, int nt, int mode, int grid) {
  if (nt <= 0) return hipSuccess;
  const dim3 G(grid > 0 && grid < nt ? grid : nt), B(MR_BLOCK);
#define MR_L1(NC_, BP_) hipLaunchKernelGGL((k1_stage<NC_, BP_>), G, B, 0, s, d, t, nt, mode)
  if (nc == 1) { if (bp) MR_L1(1, true); else MR_L1(1, false); }
  else if (nc == 3) { if (bp) MR_L1(3, true); else MR_L1(3, false); }
  else return hipErrorInvalidValue;
#undef MR_L1
  return hipGetLastError();
}

hipError_t mr_launch_stage2(hipStream_t s, int nc, int bp, mr_inst* d, const mr_tile2* t, int nt, int mode, int grid) {
  if (nt <= 0) return hipSuccess;
  const dim3 G(grid > 0 && grid < nt ? grid : nt), B(MR_BLOCK);
#define MR_L2(NC_, BP_) hipLaunchKernelGGL((k2_stage<NC_, BP_>), G, B, 0, s, d, t, nt, mode)
  if (nc == 1) { if (bp) MR_L2(1, true); else MR_L2(1, false); }
  else if (nc == 4) { if (bp) MR_L2(4, true); else MR_L2(4, false); }
  else return hipErrorInvalidValue;
#undef MR_L2
  return hipGetLastError();
}

hipError_t mr_launch_values(hipStream_t s, int dim, int nc, int bp, mr_inst* d, const mr_tile1* t, int nt, double* gl) {
  if (nt <= 0) return hipSuccess;
  const dim3 G(nt), B(MR_BLOCK);
  if (dim == 1) {
    if (nc == 1) { if (bp) hipLaunchKernelGGL((k1_values<1, true>), G, B, 0, s, d, t, nt, gl); else hipLaunchKernelGGL((k1_values<1, false>), G, B, 0, s, d, t, nt, gl); }
    else { if (bp) hipLaunchKernelGGL((k1_values<3, true>), G, B, 0, s, d, t, nt, gl); else hipLaunchKernelGGL((k1_values<3, false>), G, B, 0, s, d, t, nt, gl); }
  } else {
    if (nc == 1) { if (bp) hipLaunchKernelGGL((k2_values<1, true>), G, B, 0, s, d, t, nt, gl); else hipLaunchKernelGGL((k2_values<1, false>), G, B, 0, s, d, t, nt, gl); }
    else { if (bp) hipLaunchKernelGGL((k2_values<4, true>), G, B, 0, s, d, t, nt, gl); else hipLaunchKernelGGL((k2_values<4, false>), G, B, 0, s, d, t, nt, gl); }
  }
  return hipGetLastError();
}

}  /* extern "C" */
