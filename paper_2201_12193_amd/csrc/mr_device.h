/* Device building blocks of the MR-HWENO operator (gfx950, FP64).
 *
 * Reconstruction (Step 1 of the 1D and 2D reconstruction algorithms),
 * nonlinear weights, physical fluxes, HLLC and Lax-Friedrichs numerical
 * fluxes, and ghost-cell indexing.  The linear parts (least-squares maps,
 * smoothness-indicator quadratic forms, Gauss-Lobatto evaluation) come from
 * recon_gen.h.
 */
#pragma once
#include <hip/hip_runtime.h>
#include "mr_types.h"

/* Constant table of the generated reconstruction code (the FP64 constants
 * that an instruction cannot encode).  A translation unit that defines
 * MR_KT_IN_LDS copies it into LDS once per work group (mr_kt_fill) and reads
 * it from there, which keeps the constants out of the scalar registers of
 * its large kernels; elsewhere the entries fold into literals.  The table's
 * 256-byte alignment makes the compiler place it before the kernels' own
 * LDS blocks, at offsets that fit the immediate offset field of an LDS
 * read (above 64 KiB every constant load needed its address in a VGPR). */
#define MR_KT_MAX 128
#if defined(__HIP_DEVICE_COMPILE__) && defined(MR_KT_IN_LDS)
#define MR_KT(i) (mr_kt_lds[i])
#define MR_KT_DECLARE                                                   \
  static __constant__ double mr_kt_dev[MR_NKT + 1] = {MR_KT_VALUES};    \
  static __shared__ __attribute__((aligned(256))) double mr_kt_lds[MR_KT_MAX];
#else
#define MR_KT(i) (mr_kt_lit[i])
#define MR_KT_DECLARE static constexpr double mr_kt_lit[MR_NKT + 1] = {MR_KT_VALUES};
#endif
#include "recon_gen.h"
static_assert(MR_NKT <= MR_KT_MAX, "constant table larger than its LDS slot");

#if defined(__HIP_DEVICE_COMPILE__) && defined(MR_KT_IN_LDS)
/* copy the constant table into LDS; call at kernel entry by every thread */
__device__ __forceinline__ void mr_kt_fill() {
  for (int i = threadIdx.x; i < MR_NKT; i += blockDim.x) mr_kt_lds[i] = mr_kt_dev[i];
  __syncthreads();
}
#else
__device__ __forceinline__ void mr_kt_fill() {}
#endif

#define MR_INL __device__ __forceinline__
/* reconstruction and flux helpers also compile for the host, so that the
   kernel arithmetic can be exercised in a CPU build */
#define MR_HD __host__ __device__ __forceinline__

/* Gauss-Lobatto weights and nodes on [-1/2, 1/2], eq. (F). */
#define MR_W0 (1.0 / 12.0)
#define MR_W1 (5.0 / 12.0)
#define MR_S5 0x1.c9f25c5bfedd9p-3 /* sqrt(5)/10 */

MR_INL double glw(int k) { return (k == 0 || k == 3) ? MR_W0 : MR_W1; }
MR_INL double gln(int k) {
  return k == 0 ? -0.5 : (k == 1 ? -MR_S5 : (k == 2 ? MR_S5 : 0.5));
}

/* ------------------------------------------------------------------ ghosts */
/* Index of the interior cell whose moments cell i (possibly outside
 * [0, n)) takes under the boundary conditions bcs (kind of the low side in
 * bits 0-1, of the high side in bits 2-3), with *kind set to 1 for a
 * transmissive ghost (average copied, first moments zero) and 2 for a
 * reflective one (mirror image across the wall; see mr_refl_flip); left
 * alone for interior cells and periodic images.  Offsets up to one period
 * either side are folded; anything further is clamped (such cells never
 * feed an output). */
MR_INL int mr_fold(int i, int n, int bcs, int* kind) {
  if (i >= 0 && i < n) return i;
  const int bc = i < 0 ? (bcs & 3) : ((bcs >> 2) & 3);
  if (bc == 0) {
    if (i < 0) i += n;
    else i -= n;
  } else if (bc == 1) {
    *kind = 1;
  } else {
    *kind = 2;
    i = i < 0 ? -1 - i : 2 * n - 1 - i;
  }
  return i < 0 ? 0 : (i >= n ? n - 1 : i);
}

/* Mirror image across a wall normal to axis a (0 = x, 1 = y): the momentum
 * along the normal (component 1 + a) and the first moment along the normal
 * (moment 1 + a) change sign, so moment m of component c flips when exactly
 * one of the two holds. */
MR_HD bool mr_refl_flip(int c, int m, int a) { return (c == 1 + a) != (m == 1 + a); }

/* Face f (between cells f-1 and f) of an axis of n cells is a reflective
 * wall.  Its two traces carry opposite normal velocities, so their average
 * is exactly zero: the KXRCF test never counts it as an inflow face (the
 * computed average would only hold a rounding residue of either sign). */
MR_INL bool mr_wall(int f, int n, int bcs) {
  return (f == 0 && (bcs & 3) == 2) || (f == n && ((bcs >> 2) & 3) == 2);
}

/* 1/x for a positive (or negative) normal x of moderate size: the hardware
 * reciprocal estimate refined by two Newton steps (within about one ulp of
 * the correctly rounded value), without the range scaling and special-case
 * handling of a full division, which these arguments do not need (x = 0
 * gives NaN instead of infinity). */
MR_HD double mr_rcp(double x) {
#ifdef __HIP_DEVICE_COMPILE__
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
#else
  return 1.0 / x;
#endif
}

/* TVB minmod indicator (Remark 2's alternative): does the modified minmod
 * m~(a, dp, dm) = (|a| <= mh2 ? a : minmod(a, dp, dm)) change the face
 * deviation a?  minmod returns a itself exactly when the three arguments
 * share a's sign and |a| is the smallest, so no value is compared for
 * equality. */
MR_HD bool mr_tvb_changes(double a, double dp, double dm, double mh2) {
  if (fabs(a) <= mh2) return false;
  const bool same = (a > 0.0 && dp > 0.0 && dm > 0.0) || (a < 0.0 && dp < 0.0 && dm < 0.0);
  return !(same && fabs(a) <= fabs(dp) && fabs(a) <= fabs(dm));
}

/* ------------------------------------------------------------ nonlinear weights */
/* 1D Step 1 for one component, data on cells i-1, i, i+1 -> 4 GL values. */
template <bool BETA_P>
MR_HD void mr_recon1d(double um, double u0, double up, double vm, double v0, double vp,
                       const mr_wconst& W, double out[4]) {
  double q2[3], q3[4], q4[6];
  mr1_maps(um, u0, up, vm, v0, vp, q2, q3, q4);
  double b2, b3, b4;
  if (!BETA_P) {
    b2 = mr1_beta_k2(q2);
    b3 = mr1_beta_k3(q3);
    b4 = mr1_beta_k5(q4);
  } else {
    /* p_l = (S_l q_l - S_{l-1} q_{l-1}) / gbar_l, eq. (p) */
    double p2[3], p3[4], p4[6];
    for (int k = 0; k < 3; ++k) p2[k] = W.sg[1] * q2[k] - (k == 0 ? W.sgn[0] * u0 : 0.0);
    for (int k = 0; k < 4; ++k) p3[k] = W.sg[2] * q3[k] - (k < 3 ? W.sgn[1] * q2[k] : 0.0);
    for (int k = 0; k < 6; ++k) p4[k] = W.sg[3] * q4[k] - (k < 4 ? W.sgn[2] * q3[k] : 0.0);
    b2 = mr1_beta_k2(p2);
    b3 = mr1_beta_k3(p3);
    b4 = mr1_beta_k5(p4);
  }
  /* beta_1 from the two one-sided linear fits, eqs. (q1-LR)-(beta1).
     With d = beta + eps, gamma (1 + tau/d) normalised over the set equals
     gamma (d + tau) prod_{other} d normalised: one division per set. */
  const double dL = u0 - um, dR = up - u0;
  const double bL = dL * dL, bR = dR * dR;
  const double tdiff = bR - bL;
  const double tau1 = tdiff * tdiff;
  const double eL = bL + W.eps, eR = bR + W.eps;
  const double aL = (eL + tau1) * eR, aR = (eR + tau1) * eL;
  const double dn = (aL * dL + aR * dR) / (aL + aR);
  const double b1 = dn * dn;
  /* eqs. (tau4), (non-linear-weight) */
  double tau4 = (fabs(b4 - b1) + fabs(b4 - b2) + fabs(b4 - b3)) * (1.0 / 3.0);
  tau4 = tau4 * tau4;
  const double d1 = b1 + W.eps, d2 = b2 + W.eps, d3 = b3 + W.eps, d4 = b4 + W.eps;
  const double p12 = d1 * d2, p34 = d3 * d4;
  const double o1 = W.g4[0] * (d1 + tau4) * (d2 * p34);
  const double o2 = W.g4[1] * (d2 + tau4) * (d1 * p34);
  const double o3 = W.g4[2] * (d3 + tau4) * (p12 * d4);
  const double o4 = W.g4[3] * (d4 + tau4) * (p12 * d3);
  const double rs = mr_rcp(o1 + o2 + o3 + o4);
  const double w1 = o1 * rs, w2 = o2 * rs, w3 = o3 * rs, w4 = o4 * rs;
  /* u = sum_l w_l p_l = sum_l c_l q_l, eq. (re-p) */
  const double c1 = w1 - w2 * W.sgn[0];
  const double c2 = w2 * W.sg[1] - w3 * W.sgn[1];
  const double c3 = w3 * W.sg[2] - w4 * W.sgn[2];
  const double c4 = w4 * W.sg[3];
  double C[6];
  C[0] = c1 * u0 + c2 * q2[0] + c3 * q3[0] + c4 * q4[0];
  C[1] = c2 * q2[1] + c3 * q3[1] + c4 * q4[1];
  C[2] = c2 * q2[2] + c3 * q3[2] + c4 * q4[2];
  C[3] = c3 * q3[3] + c4 * q4[3];
  C[4] = c4 * q4[4];
  C[5] = c4 * q4[5];
  mr1_eval(C, out);
}

/* 2D Step 1 for one component; u/v/w indexed by stencil label - 1
 * (label = 1 + (dx+1) + 3 (dy+1)).  out[k + 4 l] at (xi_k, eta_l). */
template <bool BETA_P>
MR_HD void mr_recon2d(const double u[9], const double v[9], const double w[9],
                       const mr_wconst& W, double out[16]) {
  double q2[6], q3[10], q4[21];
  mr2_maps(u, v, w, q2, q3, q4);
  double b2, b3, b4;
  if (!BETA_P) {
    b2 = mr2_beta_k2(q2);
    b3 = mr2_beta_k3(q3);
    b4 = mr2_beta_k5(q4);
  } else {
    double p2[6], p3[10], p4[21];
    for (int k = 0; k < 6; ++k) p2[k] = W.sg[1] * q2[k] - (k == 0 ? W.sgn[0] * u[4] : 0.0);
    for (int k = 0; k < 10; ++k) p3[k] = W.sg[2] * q3[k] - (k < 6 ? W.sgn[1] * q2[k] : 0.0);
    for (int k = 0; k < 21; ++k) p4[k] = W.sg[3] * q4[k] - (k < 10 ? W.sgn[2] * q3[k] : 0.0);
    b2 = mr2_beta_k2(p2);
    b3 = mr2_beta_k3(p3);
    b4 = mr2_beta_k5(p4);
  }
  /* beta_1 from the four three-cell linear fits, eqs. (2D-q1-1234)-(2D-beta1) */
  const double u5 = u[4];
  const double gxl = u5 - u[3], gxr = u[5] - u5, gyb = u5 - u[1], gyt = u[7] - u5;
  const double xl2 = gxl * gxl, xr2 = gxr * gxr, yb2 = gyb * gyb, yt2 = gyt * gyt;
  const double e11 = xl2 + yt2, e12 = xr2 + yt2, e13 = xr2 + yb2, e14 = xl2 + yb2;
  double tau1 = (fabs(e11 - e12) + fabs(e11 - e13) + fabs(e11 - e14) + fabs(e12 - e13) +
                 fabs(e12 - e14) + fabs(e13 - e14)) * (1.0 / 6.0);
  tau1 = tau1 * tau1;
  /* normalised 1/4 (1 + tau1 / d_k) with one division (see the 1D case) */
  const double f1 = e11 + W.eps, f2 = e12 + W.eps, f3 = e13 + W.eps, f4 = e14 + W.eps;
  const double r12 = f1 * f2, r34 = f3 * f4;
  const double a11 = (f1 + tau1) * (f2 * r34);
  const double a12 = (f2 + tau1) * (f1 * r34);
  const double a13 = (f3 + tau1) * (r12 * f4);
  const double a14 = (f4 + tau1) * (r12 * f3);
  const double ra = mr_rcp(a11 + a12 + a13 + a14);
  const double gx = ((a11 + a14) * gxl + (a12 + a13) * gxr) * ra;
  const double gy = ((a11 + a12) * gyt + (a13 + a14) * gyb) * ra;
  const double b1 = gx * gx + gy * gy;
  double tau4 = (fabs(b4 - b1) + fabs(b4 - b2) + fabs(b4 - b3)) * (1.0 / 3.0);
  tau4 = tau4 * tau4;
  const double d1 = b1 + W.eps, d2 = b2 + W.eps, d3 = b3 + W.eps, d4 = b4 + W.eps;
  const double p12 = d1 * d2, p34 = d3 * d4;
  const double o1 = W.g4[0] * (d1 + tau4) * (d2 * p34);
  const double o2 = W.g4[1] * (d2 + tau4) * (d1 * p34);
  const double o3 = W.g4[2] * (d3 + tau4) * (p12 * d4);
  const double o4 = W.g4[3] * (d4 + tau4) * (p12 * d3);
  const double rs = mr_rcp(o1 + o2 + o3 + o4);
  const double w1 = o1 * rs, w2 = o2 * rs, w3 = o3 * rs, w4 = o4 * rs;
  const double c1 = w1 - w2 * W.sgn[0];
  const double c2 = w2 * W.sg[1] - w3 * W.sgn[1];
  const double c3 = w3 * W.sg[2] - w4 * W.sgn[2];
  const double c4 = w4 * W.sg[3];
  double C[21];
  C[0] = c1 * u5 + c2 * q2[0] + c3 * q3[0] + c4 * q4[0];
#pragma unroll
  for (int k = 1; k < 6; ++k) C[k] = c2 * q2[k] + c3 * q3[k] + c4 * q4[k];
#pragma unroll
  for (int k = 6; k < 10; ++k) C[k] = c3 * q3[k] + c4 * q4[k];
#pragma unroll
  for (int k = 10; k < 21; ++k) C[k] = c4 * q4[k];
  mr2_eval(C, out);
}

/* ------------------------------------------------------------------ fluxes */
/* Euler pressure; NC = 3 (1D) or 4 (2D). */
template <int NC>
MR_INL double mr_pressure(const double* u, double gam) {
  double m2 = u[1] * u[1];
  if (NC == 4) m2 += u[2] * u[2];
  return (gam - 1.0) * (u[NC - 1] - 0.5 * m2 / u[0]);
}

/* physical Euler flux in direction D (0 = x, 1 = y), eqs. (1D-Euler), (2D-Euler) */
template <int NC, int D>
MR_HD void mr_euler_flux(const double* u, double gam, double* f) {
  const double r = mr_rcp(u[0]);
  const double vn = u[1 + D] * r;
  double m2 = u[1] * u[1];
  if (NC == 4) m2 += u[2] * u[2];
  const double p = (gam - 1.0) * (u[NC - 1] - 0.5 * m2 * r);
  f[0] = u[1 + D];
  f[1] = u[1] * vn;
  if (NC == 4) f[2] = u[2] * vn;
  f[1 + D] += p;
  f[NC - 1] = vn * (u[NC - 1] + p);
}

/* physical fluxes f (x) and g (y) of the 2D Euler equations at one point,
 * given r = 1/rho */
MR_HD void mr_euler_fg_r(const double* u, double r, double gam, double* f, double* g) {
  const double vx = u[1] * r, vy = u[2] * r;
  const double p = (gam - 1.0) * (u[3] - 0.5 * (u[1] * u[1] + u[2] * u[2]) * r);
  f[0] = u[1]; f[1] = u[1] * vx + p; f[2] = u[2] * vx; f[3] = vx * (u[3] + p);
  g[0] = u[2]; g[1] = u[1] * vy; g[2] = u[2] * vy + p; g[3] = vy * (u[3] + p);
}

MR_HD void mr_euler_fg(const double* u, double gam, double* f, double* g) {
  mr_euler_fg_r(u, mr_rcp(u[0]), gam, f, g);
}

/* 1/a, 1/b, 1/c, 1/d with one division (positive, moderate arguments) */
MR_HD void mr_recip4(double a, double b, double c, double d, double* r) {
  const double ab = a * b, cd = c * d;
  const double inv = mr_rcp(ab * cd);
  const double icd = ab * inv, iab = cd * inv;   /* 1/(cd), 1/(ab) */
  r[0] = b * iab;
  r[1] = a * iab;
  r[2] = d * icd;
  r[3] = c * icd;
}

/* Square root of a positive normal x >= 2^-767: Goldschmidt iteration from
 * the hardware reciprocal-square-root estimate (two corrections), i.e. the
 * usual FP64 sequence without its range scaling and special-case selects,
 * which this range does not need.  Zero, negative or non-finite x give NaN
 * (a state reaching them is non-physical and is caught as such). */
MR_HD double mr_sqrtp(double x) {
#ifdef __HIP_DEVICE_COMPILE__
  const double r = __builtin_amdgcn_rsq(x);
  double g = x * r, h = 0.5 * r;
  const double e = fma(-h, g, 0.5);
  g = fma(g, e, g);
  h = fma(h, e, h);
  double d = fma(-g, g, x);
  g = fma(d, h, g);
  d = fma(-g, g, x);
  return fma(d, h, g);
#else
  return sqrt(x);
#endif
}

/* HLLC flux of eqs. (f_HLLC), (COEF), (uLR_) with the printed PVRS star
 * estimates; in 2D the normal direction D plays the role of mu and the
 * tangential momentum is carried in the star state.  Branches in the order
 * 0 <= sL, 0 <= s*, 0 <= sR, else. */
template <int NC, int D>
MR_HD void mr_hllc(const double* uL, const double* uR, double gam, double* f) {
  constexpr int N = 1 + D;
  constexpr int T = (NC == 4) ? 2 - D : 1;
  const double rL = uL[0], rR = uR[0];
  /* 1/rho_L and 1/rho_R from one division */
  const double irLR = mr_rcp(rL * rR);
  const double irL = rR * irLR, irR = rL * irLR;
  const double muL = uL[N] * irL, muR = uR[N] * irR;
  double m2L = uL[1] * uL[1], m2R = uR[1] * uR[1];
  if (NC == 4) { m2L += uL[2] * uL[2]; m2R += uR[2] * uR[2]; }
  const double EL = uL[NC - 1], ER = uR[NC - 1];
  const double pL = (gam - 1.0) * (EL - 0.5 * m2L * irL);
  const double pR = (gam - 1.0) * (ER - 0.5 * m2R * irR);
  const double cL = mr_sqrtp(gam * pL * irL), cR = mr_sqrtp(gam * pR * irR);
  const double rs = 0.5 * (rL + rR), cs = 0.5 * (cL + cR);
  const double crs = cs * rs;
  /* 1/crs, 1/p_L, 1/p_R from one division */
  const double pLR = pL * pR;
  const double i3 = mr_rcp(crs * pLR);
  const double icrs = pLR * i3, ipL = crs * pR * i3, ipR = crs * pL * i3;
  const double ps = 0.5 * (pL + pR + (muL - muR) * crs);
  const double ss = 0.5 * (muL + muR + (pL - pR) * icrs);   /* s* of the printed PVRS */
  const double k1 = (gam + 1.0) / (2.0 * gam);
  const double coefL = (ps <= pL) ? 1.0 : mr_sqrtp(1.0 + k1 * (ps * ipL - 1.0));
  const double coefR = (ps <= pR) ? 1.0 : mr_sqrtp(1.0 + k1 * (ps * ipR - 1.0));
  const double sL = muL - cL * coefL, sR = muR + cR * coefR;
  /* ordered branch chain: 0 <= sL -> f_L; 0 <= s* -> f*_L; 0 <= sR -> f*_R; f_R */
  const int br = (0.0 <= sL) ? 0 : ((0.0 <= ss) ? 1 : ((0.0 <= sR) ? 2 : 3));
  const bool left = br <= 1;
  const double* uK = left ? uL : uR;
  const double sK = left ? sL : sR;
  const double muK = left ? muL : muR;
  const double rK = left ? rL : rR;
  const double irK = left ? irL : irR;
  const double pK = left ? pL : pR;
  const double EK = left ? EL : ER;
  double fK[NC];
  fK[0] = uK[N];
  fK[1] = uK[1] * muK;
  if (NC == 4) fK[2] = uK[2] * muK;
  fK[N] += pK;
  fK[NC - 1] = muK * (EK + pK);
  if (br == 0 || br == 3) {
#pragma unroll
    for (int c = 0; c < NC; ++c) f[c] = fK[c];
    return;
  }
  const double dsK = sK - muK;
  /* rho_K (s_K - mu_K) / (s_K - s*) and p_K / (rho_K (s_K - mu_K)) share one
     reciprocal */
  const double rd = rK * dsK, den = sK - ss;
  const double inv = mr_rcp(den * rd);
  const double fac = rd * rd * inv;
  double us[NC];
  us[0] = fac;
  us[N] = fac * ss;
  if (NC == 4) us[T] = fac * (uK[T] * irK);
  us[NC - 1] = fac * (EK * irK + (ss - muK) * (ss + pK * den * inv));
#pragma unroll
  for (int c = 0; c < NC; ++c) f[c] = fK[c] + sK * (us[c] - uK[c]);
}

/* Burgers' f(u) = u^2/2 with global Lax-Friedrichs. */
MR_HD double mr_lf(double a, double b, double alpha) {
  return 0.5 * (0.5 * a * a + 0.5 * b * b - alpha * (b - a));
}

/* bits <-> double for order-preserving max of non-negative doubles */
MR_INL unsigned long long mr_dbits(double x) { return (unsigned long long)__double_as_longlong(x); }
MR_INL double mr_bitsd(unsigned long long b) { return __longlong_as_double((long long)b); }
