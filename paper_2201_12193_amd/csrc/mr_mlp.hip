/* Learned troubled-cell indicator for 2D Euler: feature extraction, the
 * fused BF16-MFMA inference kernel with its KXRCF fallback, and the kernels
 * that train the network (forward, backward, Adam).
 *
 * The indicator is not part of the paper's method: it is a small network
 * trained on the KXRCF flags (eq. (KXRCF_)) of the method's own runs, used
 * in place of Step 2.1 where it is confident.  Cells whose score falls in
 * the band [band_lo, band_hi] get the KXRCF decision.
 *
 * Features of cell (x, y): moment m in {0, 1, 2} (cell average, x and y
 * first moments) of component c in {rho, rho u, rho v, E} at cell
 * (x + wx, y + wy), |wx|, |wy| <= 2, normalised by the cell's own averages:
 *   (raw - [m == 0] centre_c) * scale_c  (evaluated as one fma with the
 *   scaled centre),
 *   scale_rho = 1/rho, scale_(rho u) = scale_(rho v) = 1/(rho c), scale_E = 1/E,
 * with c the sound speed of the cell average, plus log2(h)/16.  The values
 * are computed in FP32 and rounded to BF16.  Index of a feature: f =
 * 32 kb + 8 g + j (kb < 10, g < 4, j < 8) with slot s = 8 kb + j:
 *   s < 60:        c = s / 15, m = (s / 5) % 3, wx = s % 5 - 2, wy = g - 2;
 *   60 <= s < 75:  c = g, m = (s - 60) / 5, wx = (s - 60) % 5 - 2, wy = 2;
 *   s = 75, g = 0: log2(h)/16;   every other index is 0.
 * This order lets lane group g of the MFMA operand read window row g - 2 at
 * offsets fixed at compile time. */
#include "mr_common.h"
#include "mr_mlp.h"

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef short i16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));

MR_INL f32x4 mr_mfma(bf16x8 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

/* ------------------------------------------------------------ features */
/* normalisation of a cell from its FP32 averages: scale sc[4] and the
 * scaled centre cs[c] = centre_c * sc[c] (a feature is one fma) */
MR_INL void mr_feat_norm(float rho, float mx, float my, float E, float gam, float* sc, float* cs) {
  /* hardware reciprocal and square root (1 ulp): the features are rounded
     to BF16 afterwards */
  const float r = rho > 1e-30f ? rho : 1e-30f;
  const float ir = __builtin_amdgcn_rcpf(r);
  const float p = (gam - 1.0f) * (E - 0.5f * (mx * mx + my * my) * ir);
  float c2 = gam * p * ir;
  c2 = c2 > 1e-30f ? c2 : 1e-30f;
  const float rc = __builtin_amdgcn_rcpf(r * __builtin_amdgcn_sqrtf(c2));
  sc[0] = ir;
  sc[1] = rc;
  sc[2] = rc;
  sc[3] = __builtin_amdgcn_rcpf(E > 1e-30f ? E : 1e-30f);
  cs[0] = rho * sc[0];
  cs[1] = mx * sc[1];
  cs[2] = my * sc[2];
  cs[3] = E * sc[3];
}

MR_INL float mr_feat_val(float raw, int m, float scentre, float scale) {
  return m == 0 ? fmaf(raw, scale, -scentre) : raw * scale;
}

/* slot s of lane group g -> (component, moment, wx, wy); kind 0 moment,
 * 1 log h, 2 zero */
struct mr_fslot {
  int c, m, wx, wy, kind;
};
MR_HD mr_fslot mr_feature_slot(int s, int g) {
  if (s < 60) return mr_fslot{s / 15, (s / 5) % 3, s % 5 - 2, g - 2, 0};
  if (s < 75) return mr_fslot{g, (s - 60) / 5, (s - 60) % 5 - 2, 2, 0};
  if (s == 75 && g == 0) return mr_fslot{0, 0, 0, 0, 1};
  return mr_fslot{0, 0, 0, 0, 2};
}

/* features of n interior cells (indices j*nx + i) of one instance, one
 * thread per feature; out [n][MR_KP]; an index outside the grid gives a
 * zero row */
__global__ __launch_bounds__(MR_BLOCK) void k_features(const mr_inst* insts, int inst, const int* cells, int n,
                                                      __bf16* out) {
  const long long e = (long long)blockIdx.x * MR_BLOCK + threadIdx.x;
  if (e >= (long long)n * MR_KP) return;
  const int smp = (int)(e / MR_KP), f = (int)(e % MR_KP);
  const mr_inst& I = insts[inst];
  const mr_grid g{mr_gp(I.p_in[0]), I.plane, I.nx, I.ny, I.bcx, I.bcy, 3, nullptr, 0.0};
  const int cell = cells[smp];
  if (cell < 0 || (long long)cell >= I.plane) {   /* not an interior cell */
    out[e] = (__bf16)0.0f;
    return;
  }
  const int x = cell % I.nx, y = cell / I.nx;
  const mr_fslot sl = mr_feature_slot(8 * (f / 32) + f % 8, (f / 8) % 4);
  float v = 0.0f;
  if (sl.kind == 1) {
    v = (float)(log2(I.dx) * (1.0 / 16.0));
  } else if (sl.kind == 0) {
    float sc[4], cs[4];
    mr_feat_norm((float)mr_ld(g, 0, 0, x, y), (float)mr_ld(g, 1, 0, x, y), (float)mr_ld(g, 2, 0, x, y),
                 (float)mr_ld(g, 3, 0, x, y), (float)I.gam, sc, cs);
    v = mr_feat_val((float)mr_ld(g, sl.c, sl.m, x + sl.wx, y + sl.wy), sl.m, cs[sl.c], sc[sl.c]);
  }
  out[e] = (__bf16)v;
}

/* ------------------------------------------------------------ fused inference */
/* Work item: a strip of 64 columns x `rows` rows of the extended flag range
 * [-2, n+2)^2.  The four waves of a work group take four consecutive rows
 * per sweep step; the moments of rows y-2 .. y+5 sit in an LDS ring of
 * eight FP32 rows.  Per wave and step, 64 cells in four groups of 16:
 *   layer 1: h1 (64 x 16) = W1 (64 x 320) X (320 x 16), 40 MFMAs;
 *   layer 2: h2 = W2 relu(h1 + b1), 8 MFMAs, with the contraction order
 *            permuted alike on both operands so that the layer-1
 *            accumulators serve as the B operand without a transpose;
 *   layer 3: a dot product reduced across the four lane groups.
 * Lane i of the MFMA holds A[i%16][8(i/16)+j], B[8(i/16)+j][i%16] (j < 8)
 * and receives D[4(i/16)+j][i%16] (j < 4). */
#define MR_LW 64                       /* cells per strip row              */
#define MR_LCOLS (MR_LW + 4)           /* staged columns                   */
#define MR_LRS 80                      /* LDS row stride (floats)          */
#define MR_LPL (8 * MR_LRS + 16)       /* LDS plane stride (floats)        */
struct mr_learn_lds {
  mr_learn_w w;
  float mom[12 * MR_LPL];
};

__global__ __launch_bounds__(MR_BLOCK, 2) void k2_learned(const mr_inst* __restrict__ insts, const mr_tile2* __restrict__ tiles, int ntiles,
                                                         int stage, const mr_learn_w* wg, mr_band* band, int* cnt) {
  __shared__ mr_learn_lds sh;
  const int tid = threadIdx.x, lane = tid % 64, wv = tid / 64, r = lane % 16, g = lane / 16;
  {
    const uint4* src = reinterpret_cast<const uint4*>(wg);
    uint4* dst = reinterpret_cast<uint4*>(&sh.w);
    for (int e = tid; e < (int)(sizeof(mr_learn_w) / 16); e += MR_BLOCK) dst[e] = src[e];
  }
  const bf16x8* W1 = reinterpret_cast<const bf16x8*>(sh.w.w1);
  const bf16x8* W2 = reinterpret_cast<const bf16x8*>(sh.w.w2);
  /* staging: thread (column scol, moment sm) of the first 3 x 68 threads
     loads that column and moment of every component and row */
  const int scol = tid % MR_LCOLS, sm = tid / MR_LCOLS;
  const bool stager = tid < 3 * MR_LCOLS;
  for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const mr_tile2 tl = tiles[t];
    const mr_inst& I = insts[tl.inst];
    if (stage < 3 && !I.active) continue;
    if (I.tc != 3) continue;
    const mr_grid gr{mr_gp(stage < 3 ? I.p_in[stage] : I.buf[0]), I.plane, I.nx, I.ny, I.bcx, I.bcy, 3, nullptr, 0.0};
    MR_GLB unsigned char* fl = mr_gp(I.flags[(stage == 0 || stage == 3) ? 0 : 1]);
    const int fh = I.fhalo, fex = I.fex;
    const int xs = tl.x0 - 2, ylo = tl.y0, yhi = tl.y0 + tl.rows;
    const int xend = I.nx + fh;
    const float gam = (float)I.gam, lh = (float)(log2(I.dx) * (1.0 / 16.0));
    const float blo = (float)I.band_lo, bhi = (float)I.band_hi;
    /* staging of four rows: every thread issues its loads together (into
       registers) so that their latencies overlap, then converts and stores;
       first moments of transmissive ghosts read as zero, reflective ghosts
       flip the moments mr_refl_flip names */
    int kx = 0;
    const int ii = mr_fold(xs + scol, I.nx, I.bcx, &kx);
    const bool zx = sm != 0 && kx == 1;
    const MR_GLB double* ub = gr.U + (long long)sm * I.plane + ii;
    double pf[16];
    auto fetch = [&](int row0) {
      if (!stager) return;
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) {
        int ky = 0;
        const int jj = mr_fold(row0 + rr, I.ny, I.bcy, &ky);
        const bool zero = zx || (sm != 0 && ky == 1);
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const double v = ub[(3 * c) * I.plane + (long long)jj * I.nx];
          const bool neg = (kx == 2 && mr_refl_flip(c, sm, 0)) != (ky == 2 && mr_refl_flip(c, sm, 1));
          pf[4 * rr + c] = zero ? 0.0 : (neg ? -v : v);
        }
      }
    };
    auto store = [&](int row0) {
      if (!stager) return;
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) {
        const int slot = (row0 + rr - ylo + 2) & 7;
#pragma unroll
        for (int c = 0; c < 4; ++c)
          sh.mom[(3 * c + sm) * MR_LPL + slot * MR_LRS + scol] = (float)pf[4 * rr + c];
      }
    };
    __syncthreads();
    fetch(ylo - 2);
    store(ylo - 2);   /* rows ylo-2 .. ylo+1 */
    for (int y = ylo; y < yhi; y += 4) {
      fetch(y + 2);
      store(y + 2);   /* rows y+2 .. y+5 */
      __syncthreads();
      const int Y = y + wv;
      /* LDS bases: centre row, the lane group's window row (wy = g - 2),
         and window row wy = 2 of component g */
      const int bc = ((Y - ylo + 2) & 7) * MR_LRS + r + 2;
      const int bo = ((Y - ylo + g) & 7) * MR_LRS + r + 2;
      const int b2 = ((Y - ylo + 4) & 7) * MR_LRS + r + 2 + 3 * g * MR_LPL;
      float sc[4][4], cs[4][4], scg[4], csg[4];
#pragma unroll
      for (int gi = 0; gi < 4; ++gi) {
        mr_feat_norm(sh.mom[0 * MR_LPL + bc + 16 * gi], sh.mom[3 * MR_LPL + bc + 16 * gi],
                     sh.mom[6 * MR_LPL + bc + 16 * gi], sh.mom[9 * MR_LPL + bc + 16 * gi], gam, sc[gi], cs[gi]);
        scg[gi] = g == 0 ? sc[gi][0] : (g == 3 ? sc[gi][3] : sc[gi][1]);
        csg[gi] = g == 0 ? cs[gi][0] : (g == 1 ? cs[gi][1] : (g == 2 ? cs[gi][2] : cs[gi][3]));
      }
      /* the accumulators start from the biases: lane (r, g) accumulates
         hidden units 16m + 4g + j */
      const float4* b1v4 = reinterpret_cast<const float4*>(sh.w.b1);
      const float4* b2v4 = reinterpret_cast<const float4*>(sh.w.b2);
      const float4* w3v4 = reinterpret_cast<const float4*>(sh.w.w3);
      f32x4 h[4][4];
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        const float4 bb = b1v4[4 * m + g];
#pragma unroll
        for (int gi = 0; gi < 4; ++gi) h[gi][m] = f32x4{bb.x, bb.y, bb.z, bb.w};
      }
      /* raw moment of slot s for cell group gi (LDS), 0 for the other slots */
      auto raw = [&](int s, int gi) -> float {
        if (s < 60) {
          const int c = s / 15, m = (s / 5) % 3, wx = s % 5 - 2;
          return sh.mom[(3 * c + m) * MR_LPL + bo + 16 * gi + wx];
        }
        if (s < 75) {
          const int m = (s - 60) / 5, wx = (s - 60) % 5 - 2;
          return sh.mom[m * MR_LPL + b2 + 16 * gi + wx];
        }
        return 0.0f;
      };
      /* software pipeline over (contraction block, pair of cell groups): the
         LDS reads of the next step are issued before the current step's
         conversions and MFMAs, so their latency is hidden */
      float nxt[2][8];
#pragma unroll
      for (int h2 = 0; h2 < 2; ++h2)
#pragma unroll
        for (int j = 0; j < 8; ++j) nxt[h2][j] = raw(j, h2);
#pragma unroll
      for (int kb = 0; kb < MR_KP / 32; ++kb) {
        bf16x8 a[4];
#pragma unroll
        for (int m = 0; m < 4; ++m) a[m] = W1[(kb * 4 + m) * 64 + lane];
#pragma unroll
        for (int pr = 0; pr < 2; ++pr) {
          float cur[2][8];
#pragma unroll
          for (int h2 = 0; h2 < 2; ++h2)
#pragma unroll
            for (int j = 0; j < 8; ++j) cur[h2][j] = nxt[h2][j];
          const int nkb = pr == 1 ? kb + 1 : kb, npr = pr == 1 ? 0 : 1;
          if (nkb < MR_KP / 32) {
#pragma unroll
            for (int h2 = 0; h2 < 2; ++h2)
#pragma unroll
              for (int j = 0; j < 8; ++j) nxt[h2][j] = raw(8 * nkb + j, 2 * npr + h2);
          }
#pragma unroll
          for (int h2 = 0; h2 < 2; ++h2) {
            const int gi = 2 * pr + h2;
            bf16x8 b;
#pragma unroll
            for (int j = 0; j < 8; ++j) {
              const int s = 8 * kb + j;
              float v = 0.0f;
              if (s < 60) {
                const int c = s / 15, m = (s / 5) % 3;
                v = mr_feat_val(cur[h2][j], m, cs[gi][c], sc[gi][c]);
              } else if (s < 75) {
                v = mr_feat_val(cur[h2][j], (s - 60) / 5, csg[gi], scg[gi]);
              } else if (s == 75) {
                v = g == 0 ? lh : 0.0f;
              }
              b[j] = (__bf16)v;
            }
#pragma unroll
            for (int m = 0; m < 4; ++m) h[gi][m] = mr_mfma(a[m], b, h[gi][m]);
          }
        }
      }
      /* layer 2 and 3; this lane holds hidden units 16m + 4g + j */
      float z[4];
#pragma unroll
      for (int gi = 0; gi < 4; ++gi) {
        f32x4 o[4];
#pragma unroll
        for (int m = 0; m < 4; ++m) {
          const float4 bb = b2v4[4 * m + g];
          o[m] = f32x4{bb.x, bb.y, bb.z, bb.w};
        }
#pragma unroll
        for (int kb2 = 0; kb2 < 2; ++kb2) {
          const f32x4 x = h[gi][2 * kb2], y = h[gi][2 * kb2 + 1];
          const bf16x2 p0 = __builtin_convertvector(f32x2{x[0], x[1]}, bf16x2);
          const bf16x2 p1 = __builtin_convertvector(f32x2{x[2], x[3]}, bf16x2);
          const bf16x2 p2 = __builtin_convertvector(f32x2{y[0], y[1]}, bf16x2);
          const bf16x2 p3 = __builtin_convertvector(f32x2{y[2], y[3]}, bf16x2);
          bf16x8 b = {p0[0], p0[1], p1[0], p1[1], p2[0], p2[1], p3[0], p3[1]};
          /* ReLU after the rounding (rounding keeps the sign): a negative
             BF16 is a negative int16, so a packed integer max with 0 clears
             it, two values per instruction */
          b = __builtin_bit_cast(bf16x8, __builtin_elementwise_max(__builtin_bit_cast(i16x8, b), i16x8{}));
#pragma unroll
          for (int m = 0; m < 4; ++m) o[m] = mr_mfma(W2[(kb2 * 4 + m) * 64 + lane], b, o[m]);
        }
        float zp = 0.f;
#pragma unroll
        for (int m = 0; m < 4; ++m) {
          const float4 ww = w3v4[4 * m + g];
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const float v = o[m][j];
            /* ReLU on the bit pattern: a negative float is a negative int32 */
            zp += __builtin_bit_cast(float, max(__builtin_bit_cast(int, v), 0)) * (&ww.x)[j];
          }
        }
        zp += __shfl_xor(zp, 16);
        zp += __shfl_xor(zp, 32);
        z[gi] = zp + sh.w.b3;
      }
      /* lane L decides cell x0 + L of row Y */
      const float zz = g == 0 ? z[0] : (g == 1 ? z[1] : (g == 2 ? z[2] : z[3]));
      const float sg = __builtin_amdgcn_rcpf(1.0f + __expf(-zz));
      const int x = tl.x0 + lane;
      const bool valid = Y < yhi && x < xend;
      const unsigned char f = sg > bhi ? 1 : (sg < blo ? 0 : 2);
      const long long e = (long long)(Y + fh) * fex + (x + fh);
      if (valid) fl[e] = f;
      const unsigned long long bm = __ballot(valid && f == 2);
      if (bm) {
        int base = 0;
        if (lane == 0) base = atomicAdd(&cnt[stage], __popcll(bm));
        base = __shfl(base, 0);
        if (valid && f == 2) {
          const int pre = __popcll(bm & ((1ull << lane) - 1ull));
          band[base + pre] = mr_band{tl.inst, (int)e};
        }
      }
      __syncthreads();
    }
  }
}

/* KXRCF for the cells the network left undecided (band list, count
 * cnt[stage]) in one pass: five threads per band cell compute the face data
 * (mr2_face_summary) of the cell and of its four neighbours, and the first
 * of them evaluates eq. (KXRCF_) on them as the fused indicator kernel does.
 * One launch per smoothness-indicator variant; each skips the other's cells.
 * The learned indicator takes no per-side boundary data (the library
 * rejects the combination), so its grids carry no instance for prescribed
 * ghosts. */
template <bool BP>
__global__ __launch_bounds__(MR_BLOCK) MR_OCC void k_fb_direct(const mr_inst* __restrict__ insts, const mr_band* band, const int* cnt,
                                                              int stage) {
#pragma clang fp contract(off)
  constexpr int PB = MR_BLOCK / 5;   /* band cells per block pass */
  __shared__ double fs[PB][5][9];
  const int n = cnt[stage];
  const int tid = threadIdx.x, cb = tid / 5, d = tid % 5;
  for (int base = blockIdx.x * PB; base < n; base += gridDim.x * PB) {
    const int k = base + cb;
    const bool act = tid < 5 * PB && k < n;
    mr_band b{0, 0};
    bool mine = false;
    if (act) {
      b = band[k];
      const mr_inst& I = insts[b.inst];
      mine = (I.beta_on != 0) == BP;
      if (mine) {
        const int i = b.e % I.fex - I.fhalo, j = b.e / I.fex - I.fhalo;
        const int di = d == 1 ? -1 : (d == 2 ? 1 : 0), dj = d == 3 ? -1 : (d == 4 ? 1 : 0);
        const mr_grid g{mr_gp(stage < 3 ? I.p_in[stage] : I.buf[0]), I.plane, I.nx, I.ny, I.bcx, I.bcy, 3, nullptr, 0.0};
        double f[9];
        mr2_face_summary<BP>(g, I, i + di, j + dj, f);
#pragma unroll
        for (int q = 0; q < 9; ++q) fs[cb][d][q] = f[q];
      }
    }
    __syncthreads();
    if (mine && d == 0) {
      const mr_inst& I = insts[b.inst];
      MR_GLB unsigned char* fl = mr_gp(I.flags[(stage == 0 || stage == 3) ? 0 : 1]);
      const int i = b.e % I.fex - I.fhalo, j = b.e / I.fex - I.fhalo;
      const double tb = mr_stage_time(I, stage);
      /* face data of a cell: 0..3 face averages (left, right, bottom, top),
         4..7 the normal velocities there, 8 the norm of its values */
      const double* o = fs[cb][0];
      const double* l = fs[cb][1];
      const double* r = fs[cb][2];
      const double* bo = fs[cb][3];
      const double* t = fs[cb][4];
      double J = 0.0, len = 0.0;
      const double vl = 0.5 * (o[4] + l[5]);
      if (vl > 0.0 && !mr_wall_x(I, i, j, tb)) { J += I.dy * (o[0] - l[1]); len += I.dy; }
      const double vr = 0.5 * (o[5] + r[4]);
      if (-vr > 0.0 && !mr_wall_x(I, i + 1, j, tb)) { J += I.dy * (o[1] - r[0]); len += I.dy; }
      const double vb = 0.5 * (o[6] + bo[7]);
      if (vb > 0.0 && !mr_wall_y(I, i, j, tb)) { J += I.dx * (o[2] - bo[3]); len += I.dx; }
      const double vt = 0.5 * (o[7] + t[6]);
      if (-vt > 0.0 && !mr_wall_y(I, i, j + 1, tb)) { J += I.dx * (o[3] - t[2]); len += I.dx; }
      fl[b.e] = (unsigned char)(fabs(J) > I.dx * I.dx * len * o[8]);
    }
    __syncthreads();
  }
}

/* before a step (stages 0..2) or a probe (stage 3): clear the band counts
 * of those stages */
__global__ void k_fb_reset(int* cnt, int probe) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  if (probe) cnt[3] = 0;
  else cnt[0] = cnt[1] = cnt[2] = 0;
}

/* BF16 parameter vector -> operand-ordered weights of the fused kernel */
__global__ void k_pack_weights(const __bf16* P, mr_learn_w* w) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < MR_FRAG1) {
    const int lane = e % 64, m = (e / 64) % 4, kb = e / 256, r = lane % 16, g = lane / 16;
    bf16x8 v;
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = P[MR_OFF_W1 + (16 * m + r) * MR_KP + 32 * kb + 8 * g + j];
    reinterpret_cast<bf16x8*>(w->w1)[e] = v;
  } else if (e < MR_FRAG1 + MR_FRAG2) {
    const int k = e - MR_FRAG1;
    const int lane = k % 64, m = (k / 64) % 4, kb2 = k / 256, r = lane % 16, g = lane / 16;
    bf16x8 v;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      v[j] = P[MR_OFF_W2 + (16 * m + r) * MR_NH + 32 * kb2 + 4 * g + j];
      v[4 + j] = P[MR_OFF_W2 + (16 * m + r) * MR_NH + 32 * kb2 + 16 + 4 * g + j];
    }
    reinterpret_cast<bf16x8*>(w->w2)[k] = v;
  } else if (e < MR_FRAG1 + MR_FRAG2 + MR_NH) {
    const int o = e - MR_FRAG1 - MR_FRAG2;
    w->b1[o] = (float)P[MR_OFF_B1 + o];
    w->b2[o] = (float)P[MR_OFF_B2 + o];
    w->w3[o] = (float)P[MR_OFF_W3 + o];
    if (o == 0) {
      w->b3 = (float)P[MR_OFF_B3];
      w->pad[0] = w->pad[1] = w->pad[2] = 0.0f;
    }
  }
}

/* ------------------------------------------------------------ training */
/* C[m][n] = sum_k A[m][k] B[k][n] over BF16 operands with arbitrary strides,
 * FP32 accumulation; one wave per 16 x 16 tile of C. */
__global__ __launch_bounds__(MR_BLOCK) void k_gemm_bf16(int M, int N, int K, const __bf16* A, long long sAm,
                                                       long long sAk, const __bf16* B, long long sBk, long long sBn,
                                                       float* C, long long sCm, long long sCn) {
  const int tilesN = (N + 15) / 16;
  const int tile = blockIdx.x * (MR_BLOCK / 64) + threadIdx.x / 64;
  if (tile >= ((M + 15) / 16) * tilesN) return;
  const int m0 = (tile / tilesN) * 16, n0 = (tile % tilesN) * 16;
  const int lane = threadIdx.x % 64, r = lane % 16, g = lane / 16;
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < K; k0 += 32) {
    bf16x8 a, b;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int k = k0 + 8 * g + j;
      const bool kin = k < K;
      a[j] = (kin && m0 + r < M) ? A[(long long)(m0 + r) * sAm + (long long)k * sAk] : (__bf16)0.0f;
      b[j] = (kin && n0 + r < N) ? B[(long long)k * sBk + (long long)(n0 + r) * sBn] : (__bf16)0.0f;
    }
    acc = mr_mfma(a, b, acc);
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int m = m0 + 4 * g + j, n = n0 + r;
    if (m < M && n < N) C[(long long)m * sCm + (long long)n * sCn] = acc[j];
  }
}

/* h [B][64]: h = relu(h + b) in place; optional BF16 copy */
__global__ void k_bias_relu(int Bn, float* h, const __bf16* bias, __bf16* hb) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= Bn * MR_NH) return;
  float v = h[e] + (float)bias[e % MR_NH];
  v = v > 0.f ? v : 0.f;
  h[e] = v;
  if (hb) hb[e] = (__bf16)v;
}

/* z[s] = W3 . h2[s] + b3 */
__global__ void k_out(int Bn, const float* h2, const __bf16* P, float* zc, float* z) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= Bn) return;
  float acc = 0.0f;
  for (int o = 0; o < MR_NH; ++o) acc += (float)P[MR_OFF_W3 + o] * h2[(long long)s * MR_NH + o];
  acc += (float)P[MR_OFF_B3];
  zc[s] = acc;
  z[s] = acc;
}

/* binary cross-entropy on the logit: dz = (sigmoid(z) - y) / B and the loss
 * of each sample; dh2 = dz W3, masked where h2 = 0, in BF16 */
__global__ void k_out_back(int Bn, const float* z, const float* y, const float* h2, const __bf16* P, float* dz,
                           float* loss, __bf16* d2b) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= Bn) return;
  const float zz = z[s];
  const float d = (1.0f / (1.0f + expf(-zz)) - y[s]) / (float)Bn;
  dz[s] = d;
  loss[s] = log1pf(expf(-fabsf(zz))) + fmaxf(zz, 0.f) - y[s] * zz;
  for (int o = 0; o < MR_NH; ++o) {
    const float h = h2[(long long)s * MR_NH + o];
    d2b[(long long)s * MR_NH + o] = (__bf16)(h > 0.f ? d * (float)P[MR_OFF_W3 + o] : 0.f);
  }
}

/* per-column sums over the batch, four sample partitions per column:
 *   mode 0: db2[o] = sum dz W3[o] [h2 > 0], dW3[o] = sum dz h2, db3 = sum dz
 *   mode 1: db1[h] = sum t1 [h1 > 0]                                        */
__global__ __launch_bounds__(256) void k_colsum(int Bn, int mode, const float* dz, const float* h, const float* t1,
                                               const __bf16* P, float* G) {
  __shared__ float part[3][4][MR_NH];
  const int o = threadIdx.x % MR_NH, q = threadIdx.x / MR_NH;
  float a = 0.f, b = 0.f, c = 0.f;
  const float w3 = (float)P[MR_OFF_W3 + o];
  for (int s = q; s < Bn; s += 4) {
    const float hv = h[(long long)s * MR_NH + o];
    if (mode == 0) {
      a += hv > 0.f ? dz[s] * w3 : 0.f;
      b += dz[s] * hv;
      c += dz[s];
    } else {
      a += hv > 0.f ? t1[(long long)s * MR_NH + o] : 0.f;
    }
  }
  part[0][q][o] = a;
  part[1][q][o] = b;
  part[2][q][o] = c;
  __syncthreads();
  if (q == 0) {
    a = part[0][0][o] + part[0][1][o] + part[0][2][o] + part[0][3][o];
    b = part[1][0][o] + part[1][1][o] + part[1][2][o] + part[1][3][o];
    c = part[2][0][o] + part[2][1][o] + part[2][2][o] + part[2][3][o];
    if (mode == 0) {
      G[MR_OFF_B2 + o] = a;
      G[MR_OFF_W3 + o] = b;
      if (o == 0) G[MR_OFF_B3] = c;
      if (o < MR_NPARAM - MR_OFF_B3 - 1) G[MR_OFF_B3 + 1 + o] = 0.f;
    } else {
      G[MR_OFF_B1 + o] = a;
    }
  }
}

/* dh1 = t1 masked where h1 = 0, in BF16 */
__global__ void k_relu_back(int Bn, const float* t1, const float* h1, __bf16* d1b) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= Bn * MR_NH) return;
  d1b[e] = (__bf16)(h1[e] > 0.f ? t1[e] : 0.f);
}

/* Adam on the FP32 master parameters, refreshing the BF16 copy */
__global__ void k_adam(int n, float* w, __bf16* wb, const float* g, float* m, float* v, float lr, float b1,
                       float b2, float eps, float c1, float c2) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const float gg = g[e];
  const float mm = b1 * m[e] + (1.f - b1) * gg;
  const float vv = b2 * v[e] + (1.f - b2) * gg * gg;
  m[e] = mm;
  v[e] = vv;
  const float ww = w[e] - lr * (mm / c1) / (sqrtf(vv / c2) + eps);
  w[e] = ww;
  wb[e] = (__bf16)ww;
}

/* activation cache of one batch */
struct mr_mlp_cache {
  float *h1, *h2, *z, *dz, *t1;
  __bf16 *h1b, *d2b, *d1b;
  size_t bytes;
};
static size_t mr_al(size_t x) { return (x + 255) & ~size_t(255); }
static mr_mlp_cache mr_mlp_cache_at(void* base, int Bn) {
  mr_mlp_cache C;
  char* p = (char*)base;
  size_t off = 0;
  auto take = [&](size_t bytes) { char* q = p ? p + off : nullptr; off += mr_al(bytes); return q; };
  const size_t B = (size_t)Bn;
  C.h1 = (float*)take(4 * B * MR_NH);
  C.h2 = (float*)take(4 * B * MR_NH);
  C.t1 = (float*)take(4 * B * MR_NH);
  C.z = (float*)take(4 * B);
  C.dz = (float*)take(4 * B);
  C.h1b = (__bf16*)take(2 * B * MR_NH);
  C.d2b = (__bf16*)take(2 * B * MR_NH);
  C.d1b = (__bf16*)take(2 * B * MR_NH);
  C.bytes = off;
  return C;
}

/* ------------------------------------------------------------ launchers */
extern "C" {

hipError_t mr_launch_fb_reset(hipStream_t s, int* cnt, int probe) {
  hipLaunchKernelGGL(k_fb_reset, dim3(1), dim3(64), 0, s, cnt, probe);
  return hipGetLastError();
}

hipError_t mr_launch_pack(hipStream_t s, const void* P, mr_learn_w* w) {
  const int n = MR_FRAG1 + MR_FRAG2 + MR_NH;
  hipLaunchKernelGGL(k_pack_weights, dim3((n + 255) / 256), dim3(256), 0, s, (const __bf16*)P, w);
  return hipGetLastError();
}

hipError_t mr_launch_learned(hipStream_t s, mr_inst* d, const mr_tile2* t, int nt, int stage, const mr_learn_w* w,
                             mr_band* band, int* cnt, int grid) {
  if (nt <= 0) return hipSuccess;
  const int G = grid > 0 && grid < nt ? grid : nt;
  hipLaunchKernelGGL(k2_learned, dim3(G), dim3(MR_BLOCK), 0, s, d, t, nt, stage, w, band, cnt);
  return hipGetLastError();
}

hipError_t mr_launch_fallback(hipStream_t s, mr_inst* d, const mr_band* band, int* cnt, int stage, int grid,
                              int any_bp) {
  hipLaunchKernelGGL(k_fb_direct<false>, dim3(grid), dim3(MR_BLOCK), 0, s, d, band, cnt, stage);
  if (any_bp) hipLaunchKernelGGL(k_fb_direct<true>, dim3(grid), dim3(MR_BLOCK), 0, s, d, band, cnt, stage);
  return hipGetLastError();
}

hipError_t mr_launch_features(hipStream_t s, const mr_inst* d, int inst, const int* cells, int n, void* out) {
  if (n <= 0) return hipSuccess;
  const long long tot = (long long)n * MR_KP;
  hipLaunchKernelGGL(k_features, dim3((unsigned)((tot + MR_BLOCK - 1) / MR_BLOCK)), dim3(MR_BLOCK), 0, s, d, inst,
                     cells, n, (__bf16*)out);
  return hipGetLastError();
}

static hipError_t gemm(hipStream_t s, int M, int N, int K, const __bf16* A, long long sAm, long long sAk,
                       const __bf16* B, long long sBk, long long sBn, float* C, long long sCm, long long sCn) {
  const int tiles = ((M + 15) / 16) * ((N + 15) / 16);
  hipLaunchKernelGGL(k_gemm_bf16, dim3((tiles + 3) / 4), dim3(MR_BLOCK), 0, s, M, N, K, A, sAm, sAk, B, sBk, sBn,
                     C, sCm, sCn);
  return hipGetLastError();
}

size_t mr_mlp_cache_bytes(int batch) { return batch > 0 ? mr_mlp_cache_at(nullptr, batch).bytes : 0; }

hipError_t mr_mlp_gemm(hipStream_t s, int M, int N, int K, const void* A, long long sAm, long long sAk,
                       const void* B, long long sBk, long long sBn, void* C, long long sCm, long long sCn) {
  return gemm(s, M, N, K, (const __bf16*)A, sAm, sAk, (const __bf16*)B, sBk, sBn, (float*)C, sCm, sCn);
}

hipError_t mr_mlp_forward(hipStream_t s, const void* x, const void* params, void* cache, void* z, int Bn) {
  const __bf16* X = (const __bf16*)x;
  const __bf16* P = (const __bf16*)params;
  const mr_mlp_cache C = mr_mlp_cache_at(cache, Bn);
  hipError_t e;
  const dim3 eg((Bn * MR_NH + 255) / 256), sg((Bn + 255) / 256), blk(256);
  /* h1 = X W1^T */
  if ((e = gemm(s, Bn, MR_NH, MR_KP, X, MR_KP, 1, P + MR_OFF_W1, 1, MR_KP, C.h1, MR_NH, 1)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_bias_relu, eg, blk, 0, s, Bn, C.h1, P + MR_OFF_B1, C.h1b);
  /* h2 = relu(h1) W2^T */
  if ((e = gemm(s, Bn, MR_NH, MR_NH, C.h1b, MR_NH, 1, P + MR_OFF_W2, 1, MR_NH, C.h2, MR_NH, 1)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_bias_relu, eg, blk, 0, s, Bn, C.h2, P + MR_OFF_B2, (__bf16*)nullptr);
  hipLaunchKernelGGL(k_out, sg, blk, 0, s, Bn, C.h2, P, C.z, (float*)z);
  return hipGetLastError();
}

hipError_t mr_mlp_backward(hipStream_t s, const void* x, const void* params, void* cache, const void* labels,
                           void* grads, void* loss, int Bn) {
  const __bf16* X = (const __bf16*)x;
  const __bf16* P = (const __bf16*)params;
  float* G = (float*)grads;
  const mr_mlp_cache C = mr_mlp_cache_at(cache, Bn);
  hipError_t e;
  const dim3 eg((Bn * MR_NH + 255) / 256), sg((Bn + 255) / 256), blk(256);
  hipLaunchKernelGGL(k_out_back, sg, blk, 0, s, Bn, C.z, (const float*)labels, C.h2, P, C.dz, (float*)loss, C.d2b);
  hipLaunchKernelGGL(k_colsum, dim3(1), dim3(256), 0, s, Bn, 0, C.dz, C.h2, (const float*)nullptr, P, G);
  /* dW2[o][h] = sum_s dh2[s][o] relu(h1)[s][h] */
  if ((e = gemm(s, MR_NH, MR_NH, Bn, C.d2b, 1, MR_NH, C.h1b, MR_NH, 1, G + MR_OFF_W2, MR_NH, 1)) != hipSuccess) return e;
  /* t1[s][h] = sum_o dh2[s][o] W2[o][h] */
  if ((e = gemm(s, Bn, MR_NH, MR_NH, C.d2b, MR_NH, 1, P + MR_OFF_W2, MR_NH, 1, C.t1, MR_NH, 1)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_colsum, dim3(1), dim3(256), 0, s, Bn, 1, C.dz, C.h1, C.t1, P, G);
  hipLaunchKernelGGL(k_relu_back, eg, blk, 0, s, Bn, C.t1, C.h1, C.d1b);
  /* dW1[h][f] = sum_s dh1[s][h] X[s][f] */
  if ((e = gemm(s, MR_NH, MR_KP, Bn, C.d1b, 1, MR_NH, X, MR_KP, 1, G + MR_OFF_W1, MR_KP, 1)) != hipSuccess) return e;
  return hipGetLastError();
}

hipError_t mr_mlp_adam(hipStream_t s, void* master, void* params, const void* grads, void* m, void* v, int step,
                       float lr, float beta1, float beta2, float eps) {
  const float c1 = 1.f - powf(beta1, (float)step), c2 = 1.f - powf(beta2, (float)step);
  hipLaunchKernelGGL(k_adam, dim3((MR_NPARAM + 255) / 256), dim3(256), 0, s, MR_NPARAM, (float*)master,
                     (__bf16*)params, (const float*)grads, (float*)m, (float*)v, lr, beta1, beta2, eps, c1, c2);
  return hipGetLastError();
}

}  /* extern "C" */
