/* HIP kernels of the MR-HWENO operator for gfx950 (FP64 throughout).
 *
 * One SSP-RK3 step (eq. Runge-Kutta) is the launch sequence
 *   k_reduce(0)  -> k_finalize                      (dt from U^n, CFL)
 *   per stage s = 0, 1, 2:
 *     [k_reduce(s) for Lax-Friedrichs alpha when s > 0]
 *     1D: k1_fused(s)                               (Step 2.1 and the stage in
 *                                                    one pass)
 *     2D: k2_kxrcf (Step 2.1, KXRCF) -> k2_stage(s) (Steps 1, 2.2, 2.3, fluxes,
 *                                                    residual, RK combination)
 * The one-off evaluations (residual, reconstruction, flags) run 1D Step 2.1
 * as k1_summary -> k1_flags before k1_stage / k1_values.
 * Every kernel takes a work list spanning all instances, so one launch
 * serves a whole batch of problems of different sizes.  The 2D stage and
 * KXRCF kernels live in mr_stage2d.hip.
 *
 * Modified first moments of troubled cells replace those of the stage input
 * (Step 2.2).  Within a stage they are computed from the unmodified input
 * (Jacobi); the RK combination uses the modified stage input, and the
 * modification of U^n made in the first stage is reapplied in stages two
 * and three (1D: on the fly from the stage-1 flags; 2D: the first stage
 * keeps the modified first moments of U^n).
 */
#include "mr_common.h"

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
 * run (max is exact, so the result does not depend on the order).  The
 * descriptors of up to MR_BLOCK work items (instance, base of the data,
 * cell count) are read in parallel, one per thread, into LDS first: the
 * chain item -> instance -> state pointer -> data then costs one round of
 * latencies per batch instead of one per item.  The loads of
 * MR_RED_ITEMS work items are issued together so that their latencies
 * overlap. */
#define MR_RED_ITEMS 8
__global__ __launch_bounds__(MR_BLOCK) void k_reduce(mr_inst* insts, const mr_tile1* tiles, int ntiles,
                                                     int stage, int chunk) {
#pragma clang fp contract(off)
  __shared__ double sh[2 * (MR_BLOCK / 64)];
  __shared__ unsigned long long s_base[MR_BLOCK];   /* data of the item (0: skipped) */
  __shared__ int s_inst[MR_BLOCK], s_cnt[MR_BLOCK], s_start[MR_BLOCK];
  const int t0 = blockIdx.x * chunk, t1 = min(ntiles, t0 + chunk);
  int cur = -1;
  double ax = 0.0, ay = 0.0;
  int bad = 0;
  auto flush = [&]() {
    /* publish the finished instance (uniform across the block) */
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
  };
  for (int b0 = t0; b0 < t1; b0 += MR_BLOCK) {
    const int nb = min(MR_BLOCK, t1 - b0);
    if (b0 != t0) __syncthreads();   /* the previous batch's descriptors are consumed */
    if ((int)threadIdx.x < nb) {
      const mr_tile1 tl = tiles[b0 + threadIdx.x];
      const mr_inst& I = insts[tl.inst];
      const double* U = nullptr;
      if (stage == 0) {
        if (!I.err) U = I.buf[I.cur];
      } else if (I.active && I.flux == 0) {
        U = I.p_out[stage - 1];
      }
      s_base[threadIdx.x] = U ? (unsigned long long)(U + tl.start) : 0ull;
      s_inst[threadIdx.x] = tl.inst;
      s_cnt[threadIdx.x] = tl.count;
      s_start[threadIdx.x] = tl.start;
    }
    __syncthreads();
    for (int g0 = 0; g0 < nb; g0 += MR_RED_ITEMS) {
      double u[MR_RED_ITEMS][4];
      int inst[MR_RED_ITEMS], use[MR_RED_ITEMS];
#pragma unroll
      for (int q = 0; q < MR_RED_ITEMS; ++q) {
        const int t = g0 + q;
        inst[q] = -1;
        use[q] = 0;
        if (t >= nb) continue;
        inst[q] = s_inst[t];
        const unsigned long long base = s_base[t];
        if (!base || (int)threadIdx.x >= s_cnt[t]) continue;
        const mr_inst& I = insts[inst[q]];
        if (I.stepj > 0) {   /* the step's cells carry no state */
          const int cell = s_start[t] + (int)threadIdx.x;
          if (mr_solid(I, cell % I.nx, cell / I.nx)) continue;
        }
        const MR_GLB double* U = mr_gp((const double*)base) + threadIdx.x;
        use[q] = 1;
        const long long P = I.plane;
        const int nm = I.dim + 1;
#pragma unroll
        for (int c = 0; c < 4; ++c) u[q][c] = c < I.nc ? U[(long long)c * nm * P] : 0.0;
      }
#pragma unroll
      for (int q = 0; q < MR_RED_ITEMS; ++q) {
        if (inst[q] < 0) break;
        if (inst[q] != cur) {
          if (cur >= 0) flush();
          cur = inst[q];
        }
        if (!use[q]) continue;
        const mr_inst& I = insts[inst[q]];
        if (I.flux == 0) {
          const double a = fabs(u[q][0]);
          ax = fmax(ax, a);
          ay = fmax(ay, a);
          bad |= !(a <= 1.0e300);
        } else {
          double ke = u[q][1] * u[q][1];
          if (I.nc == 4) ke += u[q][2] * u[q][2];
          const double E = I.nc == 4 ? u[q][3] : u[q][2];
          const double p = (I.gam - 1.0) * (E - 0.5 * ke / u[q][0]);
          const double cs = sqrt(I.gam * p / u[q][0]);
          const double sx = fabs(u[q][1] / u[q][0]) + cs;
          const double sy = (I.nc == 4) ? fabs(u[q][2] / u[q][0]) + cs : 0.0;
          const int b = !(u[q][0] > 0.0) || !(p > 0.0) || !(sx <= 1.0e300) || !(sy <= 1.0e300);
          bad |= b;
          if (!b) { ax = fmax(ax, sx); ay = fmax(ay, sy); }
        }
      }
    }
  }
  if (cur >= 0) flush();
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
/* KXRCF face data of the cell i (extended range [-3, nx+3)): 0 own value
 * at x_{i-1/2}, 1 at x_{i+1/2}, 2 velocity at x_{i-1/2}, 3 at x_{i+1/2},
 * 4 max |u| over the 4 GL points (Step 1 on the unmodified stage input). */
template <bool BP>
MR_INL void mr1_face_data(const mr_grid& g, const mr_inst& I, int i, double S[5]) {
  double r[4];
  double vl, vr;
  if (I.charwise) {
    /* characteristic-wise Step 1 gives all components together */
    double um[3], u0[3], up[3], vm[3], v0[3], vp[3], rr[3][4];
    for (int c = 0; c < 3; ++c) {
      um[c] = mr_ld(g, c, 0, i - 1, 0); u0[c] = mr_ld(g, c, 0, i, 0); up[c] = mr_ld(g, c, 0, i + 1, 0);
      vm[c] = mr_ld(g, c, 1, i - 1, 0); v0[c] = mr_ld(g, c, 1, i, 0); vp[c] = mr_ld(g, c, 1, i + 1, 0);
    }
    mr1_recon_sys<3, BP>(um, u0, up, vm, v0, vp, I, rr);
    for (int k = 0; k < 4; ++k) r[k] = rr[0][k];
    vl = rr[1][0] / r[0];
    vr = rr[1][3] / r[3];
  } else {
    mr_recon1d<BP>(mr_ld(g, 0, 0, i - 1, 0), mr_ld(g, 0, 0, i, 0), mr_ld(g, 0, 0, i + 1, 0),
                   mr_ld(g, 0, 1, i - 1, 0), mr_ld(g, 0, 1, i, 0), mr_ld(g, 0, 1, i + 1, 0), I.W, r);
    vl = r[0];
    vr = r[3];
    if (I.flux == 1 && I.tc != 4) {   /* the TVB test needs no velocity */
      double m[4];
      mr_recon1d<BP>(mr_ld(g, 1, 0, i - 1, 0), mr_ld(g, 1, 0, i, 0), mr_ld(g, 1, 0, i + 1, 0),
                     mr_ld(g, 1, 1, i - 1, 0), mr_ld(g, 1, 1, i, 0), mr_ld(g, 1, 1, i + 1, 0), I.W, m);
      vl = m[0] / r[0];
      vr = m[3] / r[3];
    }
  }
  double nrm = 0.0;
#pragma unroll
  for (int k = 0; k < 4; ++k) nrm = fmax(nrm, fabs(r[k]));
  S[0] = r[0];
  S[1] = r[3];
  S[2] = vl;
  S[3] = vr;
  S[4] = nrm;
}

/* Troubled-cell flag of the cell i from the face data of i-1, i, i+1
 * (sl1, sl3: entries 1, 3 of i-1; s: all of i; sr0, sr2: entries 0, 2 of
 * i+1): eq. (KXRCF) with eq. (line-integral-average), or, for tc = 4, the
 * TVB minmod test on the face deviations of the indicator variable (cell
 * averages from g).  *num, *den: the two sides of the KXRCF comparison. */
MR_INL bool mr1_flag(const mr_inst& I, const mr_grid& g, int i, double tb, double sl1, double sl3, const double* s,
                     double sr0, double sr2, double* num, double* den) {
#pragma clang fp contract(off)
  if (I.tc == 4) {
    const double ub = mr_ld(g, 0, 0, i, 0);
    const double dp = mr_ld(g, 0, 0, i + 1, 0) - ub, dm = ub - mr_ld(g, 0, 0, i - 1, 0);
    *num = *den = 0.0;
    return mr_tvb_changes(s[1] - ub, dp, dm, I.tvb_mh2) || mr_tvb_changes(ub - s[0], dp, dm, I.tvb_mh2);
  }
  const double jl = s[0] - sl1;
  const double vl = 0.5 * (s[2] + sl3);
  const double jr = s[1] - sr0;
  const double vr = 0.5 * (s[3] + sr2);
  const bool il = vl > 0.0 && !mr_wall_x(I, i, 0, tb), ir = -vr > 0.0 && !mr_wall_x(I, i + 1, 0, tb);
  const double J = jl * (il ? 1.0 : 0.0) + jr * (ir ? 1.0 : 0.0);
  *num = fabs(J);
  *den = I.dx * I.dx * s[4];
  return *num > *den;
}

/* KXRCF face data per cell over the extended range [-3, nx+3) into the
 * summary planes (plane k = entry k of mr1_face_data). */
template <bool BP, bool GB>
__global__ __launch_bounds__(MR_BLOCK) MR_OCC void k1_summary(const mr_inst* __restrict__ insts, const mr_tile1* __restrict__ tiles, int ntiles, int stage) {
  mr_kt_fill();
  for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const mr_tile1 tl = tiles[t];
    const mr_inst& I = insts[tl.inst];
    if (stage < 3 && !I.active) continue;
    if (I.tc != 1 && I.tc != 3 && I.tc != 4) continue;
    const int e = tl.start + (int)threadIdx.x;
    if (e >= tl.start + tl.count) continue;
    const int i = e - I.shalo;
    mr_grid g{mr_gp(stage < 3 ? I.p_in[stage] : I.buf[0]), I.plane, I.nx, 1, I.bcx, I.bcy, 2, GB ? &I : nullptr,
              mr_stage_time(I, stage)};
    double S5[5];
    mr1_face_data<BP>(g, I, i, S5);
    const long long SE = I.sex;
    MR_GLB double* S = mr_gp(I.summ);
#pragma unroll
    for (int k = 0; k < 5; ++k) S[k * SE + e] = S5[k];
  }
}

/* Troubled-cell flags (mr1_flag) over [-2, nx+2); tc = 0 / 2 write
 * all-zero / all-one maps. */
__global__ __launch_bounds__(MR_BLOCK) void k1_flags(const mr_inst* __restrict__ insts, const mr_tile1* __restrict__ tiles, int ntiles, int stage) {
  for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const mr_tile1 tl = tiles[t];
    const mr_inst& I = insts[tl.inst];
    if (stage < 3 && !I.active) continue;
    const int e = tl.start + (int)threadIdx.x;
    if (e >= tl.start + tl.count) continue;
    MR_GLB unsigned char* fl = mr_gp(I.flags[(stage == 0 || stage == 3) ? 0 : 1]);
    if (I.tc == 0 || I.tc == 2) { fl[e] = (unsigned char)(I.tc == 2); continue; }
    const int s = e + (I.shalo - I.fhalo);   /* same cell in the summary plane */
    const long long SE = I.sex;
    const MR_GLB double* S = mr_gp(I.summ);
    const mr_grid g{mr_gp(stage < 3 ? I.p_in[stage] : I.buf[0]), I.plane, I.nx, 1, I.bcx, I.bcy, 2, &I, mr_stage_time(I, stage)};
    const int i = e - I.fhalo;
    double own[5], num, den;
#pragma unroll
    for (int k = 0; k < 5; ++k) own[k] = S[k * SE + s];
    const bool f = mr1_flag(I, g, i, mr_stage_time(I, stage), S[1 * SE + s - 1], S[3 * SE + s - 1], own,
                            S[0 * SE + s + 1], S[2 * SE + s + 1], &num, &den);
    fl[e] = (unsigned char)f;
    if (I.tc != 4 && I.aleph && i >= 0 && i < I.nx) { I.aleph[2 * i] = num; I.aleph[2 * i + 1] = den; }
  }
}

/* Steps 1, 2.2, 2.3, fluxes, residual and RK combination of the cell x of
 * thread cs (the threads of a work group hold consecutive cells; the cell
 * of thread cs - 1 supplies the left face value), given the flags f0, fm,
 * fp of x, x - 1, x + 1; cells with `out` write their result.  Contains the
 * work group's barriers: every thread calls it. */
template <int NC, bool BP, bool GB>
MR_INL void mr1_stage_cell(const mr_inst& I, int mode, int x, bool out, int f0, int fm, int fp, double* s_tr,
                           double* s_fl) {
  const int cs = threadIdx.x;
  const int st = mode == 3 ? 0 : mode;
  const int fh = I.fhalo;
  const mr_grid g{mr_gp(I.p_in[st]), I.plane, I.nx, 1, I.bcx, I.bcy, 2, GB ? &I : nullptr, mr_stage_time(I, mode)};
  double val[NC][4], vt[NC][2];
  double um[NC], u0[NC], up[NC], vm[NC], v0[NC], vp[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    um[c] = mr_ld(g, c, 0, x - 1, 0); u0[c] = mr_ld(g, c, 0, x, 0); up[c] = mr_ld(g, c, 0, x + 1, 0);
    vm[c] = mr_ld(g, c, 1, x - 1, 0); v0[c] = mr_ld(g, c, 1, x, 0); vp[c] = mr_ld(g, c, 1, x + 1, 0);
    const double v0s = v0[c];   /* stored first moment */
    if (f0) {
      /* Steps 2.2/2.3: Step 1 again with the troubled cells' first moments modified */
      if (fm) vm[c] = mr_modified_moment(mr_ld(g, c, 0, x - 2, 0), u0[c], mr_ld(g, c, 1, x - 2, 0), v0[c]);
      vp[c] = fp ? mr_modified_moment(u0[c], mr_ld(g, c, 0, x + 2, 0), v0[c], mr_ld(g, c, 1, x + 2, 0)) : vp[c];
      v0[c] = mr_modified_moment(um[c], up[c], mr_ld(g, c, 1, x - 1, 0), mr_ld(g, c, 1, x + 1, 0));
    }
    vt[c][0] = u0[c];
    vt[c][1] = I.mod == 1 ? v0s : v0[c];   /* internal to L: the combination keeps the stored moment */
  }
  mr1_recon_sys<NC, BP>(um, u0, up, vm, v0, vp, I, val);
#pragma unroll
  for (int c = 0; c < NC; ++c) s_tr[cs * NC + c] = val[c][3];
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
    MR_GLB double* O = mr_gp(I.p_out[st]);
    const long long P = I.plane;
    const double dt = I.dt;
    const mr_grid gn{mr_gp(I.p_un), I.plane, I.nx, 1, I.bcx, I.bcy, 2, GB ? &I : nullptr, mr_stage_time(I, 0)};
    /* U^n with the stage-1 modification (stored first moments unless it persists) */
    const int f1 = (mode == 1 || mode == 2) && I.mod == 0 ? mr_flag(mr_gp(I.flags[0]), I.fex, 1, fh, x, 0) : 0;
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
}

/* 1D stage: one thread per cell of a block-sized tile; the two edge threads
 * are ring cells that only supply face values.  Flags from the flag plane
 * (k1_flags).  mode 0..2 = RK stage, mode 3 = write L(U) (input p_in[0],
 * output p_out[0]). */
template <int NC, bool BP, bool GB>
__global__ __launch_bounds__(MR_BLOCK) MR_OCC void k1_stage(const mr_inst* __restrict__ insts, const mr_tile1* __restrict__ tiles, int ntiles, int mode) {
  mr_kt_fill();
  __shared__ double s_tr[MR_BLOCK * NC];
  __shared__ double s_fl[MR_BLOCK * NC];
  const int cs = threadIdx.x;
  for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const mr_tile1 tl = tiles[t];
    const mr_inst& I = insts[tl.inst];
    if (mode < 3 && !I.active) continue;
    const MR_GLB unsigned char* fl = mr_gp(I.flags[(mode == 0 || mode == 3) ? 0 : 1]);
    const int x = tl.start - 1 + cs;
    const int fh = I.fhalo;
    const int f0 = mr_flag(fl, I.fex, 1, fh, x, 0);
    int fm = 0, fp = 0;
    if (f0) { fm = mr_flag(fl, I.fex, 1, fh, x - 1, 0); fp = mr_flag(fl, I.fex, 1, fh, x + 1, 0); }
    const bool out = cs >= 1 && cs <= MR_BLOCK - 2 && x < I.nx && x < tl.start + tl.count;
    mr1_stage_cell<NC, BP, GB>(I, mode, x, out, f0, fm, fp, s_tr, s_fl);
    __syncthreads();
  }
}

/* 1D stage with Step 2.1 in the same pass (the step's launches; the
 * one-off evaluations use k1_summary, k1_flags and k1_stage).  A work
 * group owns up to MR_BLOCK - 6 cells plus three ring cells each side,
 * one thread per cell: every thread computes the face data of its cell
 * into LDS (mr1_face_data), then its flag (mr1_flag) -- valid from the
 * second to the second-to-last thread, which covers the flags of the owned
 * cells and of their neighbours that the modification reads -- then the
 * stage (mr1_stage_cell) with those flags.  The flags of the owned cells
 * also go to the flag plane: stages 2 and 3 read back those of stage 1 for
 * U^n.  Same arithmetic as the three separate kernels. */
template <int NC, bool BP, bool GB>
__global__ __launch_bounds__(MR_BLOCK) MR_OCC void k1_fused(const mr_inst* __restrict__ insts, const mr_tile1* __restrict__ tiles, int ntiles, int mode) {
  mr_kt_fill();
  __shared__ double s_sd[5 * MR_BLOCK];
  __shared__ unsigned char s_flg[MR_BLOCK];
  __shared__ double s_tr[MR_BLOCK * NC];
  __shared__ double s_fl[MR_BLOCK * NC];
  const int cs = threadIdx.x;
  for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const mr_tile1 tl = tiles[t];
    const mr_inst& I = insts[tl.inst];
    if (!I.active) continue;
    const int x = tl.start - 3 + cs;
    const double tb = mr_stage_time(I, mode);
    const bool kx = I.tc == 1 || I.tc == 4;
    if (kx) {
      const mr_grid g{mr_gp(I.p_in[mode]), I.plane, I.nx, 1, I.bcx, I.bcy, 2, GB ? &I : nullptr, tb};
      double S5[5];
      mr1_face_data<BP>(g, I, x, S5);
#pragma unroll
      for (int k = 0; k < 5; ++k) s_sd[k * MR_BLOCK + cs] = S5[k];
    }
    __syncthreads();
    unsigned char f = I.tc == 2 ? 1 : 0;
    if (kx && cs >= 1 && cs <= MR_BLOCK - 2) {
      const mr_grid g{mr_gp(I.p_in[mode]), I.plane, I.nx, 1, I.bcx, I.bcy, 2, &I, tb};
      double own[5], num, den;
#pragma unroll
      for (int k = 0; k < 5; ++k) own[k] = s_sd[k * MR_BLOCK + cs];
      f = (unsigned char)mr1_flag(I, g, x, tb, s_sd[1 * MR_BLOCK + cs - 1], s_sd[3 * MR_BLOCK + cs - 1], own,
                                  s_sd[0 * MR_BLOCK + cs + 1], s_sd[2 * MR_BLOCK + cs + 1], &num, &den);
    }
    s_flg[cs] = f;
    const bool own_cell = cs >= 3 && x < tl.start + tl.count && x < I.nx;
    if (own_cell) mr_gp(I.flags[mode == 0 ? 0 : 1])[x + I.fhalo] = f;
    __syncthreads();
    const bool inner = cs >= 1 && cs <= MR_BLOCK - 2;
    const int f0 = inner ? s_flg[cs] : 0;
    const int fm = inner && f0 ? s_flg[cs - 1] : 0, fp = inner && f0 ? s_flg[cs + 1] : 0;
    mr1_stage_cell<NC, BP, GB>(I, mode, x, own_cell, f0, fm, fp, s_tr, s_fl);
    __syncthreads();
  }
}

/* 1D final Gauss-Lobatto values of interior cells: gl[(c*4 + k)*nx + i]. */
template <int NC, bool BP>
__global__ __launch_bounds__(MR_BLOCK) MR_OCC void k1_values(const mr_inst* __restrict__ insts, const mr_tile1* __restrict__ tiles, int ntiles, double* gl) {
  mr_kt_fill();
  for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const mr_tile1 tl = tiles[t];
    const mr_inst& I = insts[tl.inst];
    const int x = tl.start + (int)threadIdx.x;
    if (x >= tl.start + tl.count) continue;
    const mr_grid g{mr_gp(I.p_in[0]), I.plane, I.nx, 1, I.bcx, I.bcy, 2, &I, mr_stage_time(I, 3)};
    const MR_GLB unsigned char* fl = mr_gp(I.flags[0]);
    const int fh = I.fhalo;
    const int f0 = mr_flag(fl, I.fex, 1, fh, x, 0);
    const int fm = mr_flag(fl, I.fex, 1, fh, x - 1, 0), fp = mr_flag(fl, I.fex, 1, fh, x + 1, 0);
    double um[NC], u0[NC], up[NC], vm[NC], v0[NC], vp[NC], r[NC][4];
    for (int c = 0; c < NC; ++c) {
      um[c] = mr_ld(g, c, 0, x - 1, 0); u0[c] = mr_ld(g, c, 0, x, 0); up[c] = mr_ld(g, c, 0, x + 1, 0);
      vm[c] = mr_ld(g, c, 1, x - 1, 0); v0[c] = mr_ld(g, c, 1, x, 0); vp[c] = mr_ld(g, c, 1, x + 1, 0);
      if (f0) {
        if (fm) vm[c] = mr_modified_moment(mr_ld(g, c, 0, x - 2, 0), u0[c], mr_ld(g, c, 1, x - 2, 0), v0[c]);
        if (fp) vp[c] = mr_modified_moment(u0[c], mr_ld(g, c, 0, x + 2, 0), v0[c], mr_ld(g, c, 1, x + 2, 0));
        v0[c] = mr_modified_moment(um[c], up[c], mr_ld(g, c, 1, x - 1, 0), mr_ld(g, c, 1, x + 1, 0));
      }
    }
    mr1_recon_sys<NC, BP>(um, u0, up, vm, v0, vp, I, r);
    for (int c = 0; c < NC; ++c)
      for (int k = 0; k < 4; ++k) gl[(long long)(c * 4 + k) * I.plane + x] = r[c][k];
  }
}

/* ================================================================ 2D passes */
/* Flags of the 2D instances without an indicator pass (no troubled cells,
 * or all cells troubled) over [-2, n+2)^2; the KXRCF flags of 2D instances
 * come from the fused kernel k2_kxrcf, the learned ones from k2_learned. */
__global__ __launch_bounds__(MR_BLOCK) void k2_flags(const mr_inst* __restrict__ insts, const mr_tile1* __restrict__ tiles, int ntiles, int stage) {
  for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const mr_tile1 tl = tiles[t];
    const mr_inst& I = insts[tl.inst];
    if (stage < 3 && !I.active) continue;
    const int e = tl.start + (int)threadIdx.x;
    if (e >= tl.start + tl.count) continue;
    MR_GLB unsigned char* fl = mr_gp(I.flags[(stage == 0 || stage == 3) ? 0 : 1]);
    if (I.tc == 0 || I.tc == 2) fl[e] = (unsigned char)(I.tc == 2);
  }
}

template <int NC, bool BP>
__global__ __launch_bounds__(MR_BLOCK) MR_OCC void k2_values(const mr_inst* __restrict__ insts, const mr_tile1* __restrict__ tiles, int ntiles, double* gl) {
  mr_kt_fill();
  for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const mr_tile1 tl = tiles[t];
    const mr_inst& I = insts[tl.inst];
    const int e = tl.start + (int)threadIdx.x;
    if (e >= tl.start + tl.count) continue;
    const int x = e % I.nx, y = e / I.nx;
    const mr_grid g{mr_gp(I.p_in[0]), I.plane, I.nx, I.ny, I.bcx, I.bcy, 3, &I, mr_stage_time(I, 3)};
    if (NC == 4 && I.charwise) {
      /* characteristic-wise: the set of the x direction */
      double val[4][16];
      mr2_cell_values_ch<BP, 0>(g, I, mr_gp(I.flags[0]), x, y, val);
      for (int c = 0; c < 4; ++c)
        for (int p = 0; p < 16; ++p) gl[(long long)(c * 16 + p) * I.plane + e] = val[c][p];
      continue;
    }
    for (int c = 0; c < NC; ++c) {
      double val[16], a, b, d;
      mr2_cell_values<BP>(g, I, mr_gp(I.flags[0]), c, x, y, val, &a, &b, &d);
      for (int p = 0; p < 16; ++p) gl[(long long)(c * 16 + p) * I.plane + e] = val[p];
    }
  }
}

/* ============================================================ host launchers */
extern "C" {

hipError_t mr_launch_reduce(hipStream_t s, mr_inst* d, const mr_tile1* t, int nt, int stage) {
  if (nt <= 0) return hipSuccess;
  /* few enough work groups that the per-instance atomics do not contend */
  const int chunk = nt > 512 ? (nt + 511) / 512 : 1;
  const int grid = (nt + chunk - 1) / chunk;
  hipLaunchKernelGGL(k_reduce, dim3(grid), dim3(MR_BLOCK), 0, s, d, t, nt, stage, chunk);
  return hipGetLastError();
}

hipError_t mr_launch_finalize(hipStream_t s, mr_inst* d, int n, int probe) {
  hipLaunchKernelGGL(k_finalize, dim3((n + 63) / 64), dim3(64), 0, s, d, n, probe);
  return hipGetLastError();
}

/* gb: some instance of the list has ghosts that hold prescribed data (the
   variants without that code run everything else) */
hipError_t mr_launch_summary(hipStream_t s, int dim, int bp, int gb, mr_inst* d, const mr_tile1* t, int nt, int stage) {
  if (nt <= 0) return hipSuccess;
  if (dim != 1) return hipErrorInvalidValue;   /* 2D: k2_kxrcf */
  const dim3 G(nt), B(MR_BLOCK);
  if (bp) {
    if (gb) hipLaunchKernelGGL((k1_summary<true, true>), G, B, 0, s, d, t, nt, stage);
    else hipLaunchKernelGGL((k1_summary<true, false>), G, B, 0, s, d, t, nt, stage);
  } else {
    if (gb) hipLaunchKernelGGL((k1_summary<false, true>), G, B, 0, s, d, t, nt, stage);
    else hipLaunchKernelGGL((k1_summary<false, false>), G, B, 0, s, d, t, nt, stage);
  }
  return hipGetLastError();
}

hipError_t mr_launch_flags(hipStream_t s, int dim, mr_inst* d, const mr_tile1* t, int nt, int stage) {
  if (nt <= 0) return hipSuccess;
  if (dim == 1) hipLaunchKernelGGL(k1_flags, dim3(nt), dim3(MR_BLOCK), 0, s, d, t, nt, stage);
  else hipLaunchKernelGGL(k2_flags, dim3(nt), dim3(MR_BLOCK), 0, s, d, t, nt, stage);
  return hipGetLastError();
}

hipError_t mr_launch_stage1(hipStream_t s, int nc, int bp, int gb, mr_inst* d, const mr_tile1* t, int nt, int mode,
                            int grid) {
  if (nt <= 0) return hipSuccess;
  const dim3 G(grid > 0 && grid < nt ? grid : nt), B(MR_BLOCK);
#define MR_L1(NC_, BP_)                                                                  \
  do {                                                                                   \
    if (gb) hipLaunchKernelGGL((k1_stage<NC_, BP_, true>), G, B, 0, s, d, t, nt, mode);  \
    else hipLaunchKernelGGL((k1_stage<NC_, BP_, false>), G, B, 0, s, d, t, nt, mode);    \
  } while (0)
  if (nc == 1) { if (bp) MR_L1(1, true); else MR_L1(1, false); }
  else if (nc == 3) { if (bp) MR_L1(3, true); else MR_L1(3, false); }
  else return hipErrorInvalidValue;
#undef MR_L1
  return hipGetLastError();
}

/* the step's 1D stage with Step 2.1 (k1_fused), modes 0..2; tiles of at
   most MR_BLOCK - 6 cells */
hipError_t mr_launch_fused1(hipStream_t s, int nc, int bp, int gb, mr_inst* d, const mr_tile1* t, int nt, int mode) {
  if (nt <= 0) return hipSuccess;
  if (mode < 0 || mode > 2) return hipErrorInvalidValue;
  const dim3 G(nt), B(MR_BLOCK);
#define MR_LF(NC_, BP_)                                                                  \
  do {                                                                                   \
    if (gb) hipLaunchKernelGGL((k1_fused<NC_, BP_, true>), G, B, 0, s, d, t, nt, mode);  \
    else hipLaunchKernelGGL((k1_fused<NC_, BP_, false>), G, B, 0, s, d, t, nt, mode);    \
  } while (0)
  if (nc == 1) { if (bp) MR_LF(1, true); else MR_LF(1, false); }
  else if (nc == 3) { if (bp) MR_LF(3, true); else MR_LF(3, false); }
  else return hipErrorInvalidValue;
#undef MR_LF
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
