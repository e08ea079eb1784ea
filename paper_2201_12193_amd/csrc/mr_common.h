/* Helpers shared by the kernel translation units of the MR-HWENO library. */
#pragma once
#include "mr_device.h"

#define MR_BLOCK 256
/* occupancy target for the reconstruction kernels: the compiler schedules
   for at most 512 / MR_WAVES VGPRs per lane instead of the whole file */
#ifndef MR_WAVES
#define MR_WAVES 2
#endif
#define MR_OCC __attribute__((amdgpu_waves_per_eu(MR_WAVES)))

/* =================================================================== helpers */
/* Global-memory view of a pointer taken from an instance descriptor.  The
 * compiler cannot infer the address space of a pointer loaded from memory
 * and would access it with flat instructions, which also count against the
 * LDS wait counter: every LDS wait would then wait for the HBM loads in
 * flight as well. */
#define MR_GLB __attribute__((address_space(1)))
template <class T>
MR_INL MR_GLB T* mr_gp(T* p) { return (MR_GLB T*)p; }

/* Time of the boundary data in stage s of the step (t^n, t^n + dt,
 * t^n + dt/2), or the current time for a one-off evaluation (s = 3). */
MR_INL double mr_stage_time(const mr_inst& I, int s) {
#pragma clang fp contract(off)
  return s == 0 ? I.t_prev : (s == 1 ? I.t_prev + I.dt : (s == 2 ? I.t_prev + 0.5 * I.dt : I.t));
}

/* Area and first moments (of xi and eta) of the part of the reference cell
 * [-1/2, 1/2]^2 where a xi + b eta < c.  The polygon formulas are sums over
 * its directed edges: the parts of the square's edges inside the
 * half-plane plus the chord from where the boundary leaves the half-plane
 * to where it comes back. */
MR_INL void mr_clip(double a, double b, double c, double* area, double* mx, double* my) {
#pragma clang fp contract(off)
  const double cx[4] = {-0.5, 0.5, 0.5, -0.5}, cy[4] = {-0.5, -0.5, 0.5, 0.5};
  double A = 0.0, X = 0.0, Y = 0.0, ox = 0.0, oy = 0.0, ix = 0.0, iy = 0.0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int l = (k + 1) & 3;
    const double fk = a * cx[k] + b * cy[k] - c, fl = a * cx[l] + b * cy[l] - c;
    const bool ink = fk < 0.0, inl = fl < 0.0;
    double x0 = cx[k], y0 = cy[k], x1 = cx[l], y1 = cy[l];
    if (ink != inl) {
      const double r = fk / (fk - fl);
      const double xs = cx[k] + r * (cx[l] - cx[k]), ys = cy[k] + r * (cy[l] - cy[k]);
      if (ink) { x1 = xs; y1 = ys; ox = xs; oy = ys; }   /* leaves the half-plane */
      else { x0 = xs; y0 = ys; ix = xs; iy = ys; }       /* comes back           */
    }
    if (ink || inl) {
      const double cr = x0 * y1 - x1 * y0;
      A += cr; X += (x0 + x1) * cr; Y += (y0 + y1) * cr;
    }
  }
  const double cr = ox * iy - ix * oy;   /* the chord (zero if the cell is not cut) */
  A += cr; X += (ox + ix) * cr; Y += (oy + iy) * cr;
  *area = A / 2.0;
  *mx = X / 6.0;
  *my = Y / 6.0;
}

/* Prescribed data of the ghost cell (i, j) at time t.  The bottom and top
 * sides may carry a front x < s0 + st t + sn y (a straight front moving at
 * constant speed).  On an inflow side the cells it cuts hold the exact
 * moments of the two-state field (`spre` before the front, the inflow
 * state beyond); before a folded side (transmissive, reflective) the ghost
 * holds `spre` if its centre lies before the front.  Left and right inflow
 * sides hold their state; the bottom and top sides take precedence in the
 * corners.  A constant state has zero first moments. */
MR_INL bool mr_presc_any(const mr_inst& I, int i, int j, double t) {
#pragma clang fp contract(off)
  if (I.dim == 2 && (j < 0 || j >= I.ny)) {
    const int s = j < 0 ? 2 : 3;
    if ((I.pres >> s) & 1) {
      if (I.skind[s] == 3) return true;
      const double xc = I.x0 + (i + 0.5) * I.dx, yc = I.y0 + (j + 0.5) * I.dy;
      if (xc < I.ssplit[s][0] + I.ssplit[s][1] * t + I.ssplit[s][2] * yc) return true;
    }
  }
  if (i < 0 || i >= I.nx) {
    const int s = i < 0 ? 0 : 1;
    if (((I.pres >> s) & 1) && I.skind[s] == 3) return true;
  }
  return false;
}

/* whether any cell of columns x0 .. x0+w-1 and rows y0 .. y0+nr-1 can hold
   prescribed data or read a cell of the step: a row outside [0, ny) with
   data on the bottom or top side, a column outside [0, nx) with data on the
   left or right side, or a block that reaches the step's rows and columns
   (uniform over a work group: the rows and columns of its strip; STEP =
   false: kernel variants for instances without a step) */
template <bool STEP = true>
MR_INL bool mr_presc_rows(const mr_inst& I, int x0, int w, int y0, int nr) {
  if (nr <= 0) return false;
  if (STEP && I.stepj > 0 && y0 < I.stepj && x0 + w > I.stepi) return true;
  if (!I.pres) return false;
  if ((I.pres & 12) && (y0 < 0 || y0 + nr > I.ny)) return true;
  return (I.pres & 3) && (x0 < 0 || x0 + w > I.nx);
}

/* cell (i, j) of the grid lies in the step */
MR_INL bool mr_solid(const mr_inst& I, int i, int j) {
  return I.stepj > 0 && i >= I.stepi && i < I.nx && j >= 0 && j < I.stepj;
}

/* A cell of the step read as a ghost is the mirror image of a fluid cell
 * across the step's nearest face: across the vertical face x = stepi when
 * the cell lies fewer columns into the step than rows below its top,
 * across the top y = stepj in the opposite case, across both (through the
 * corner) when the two depths are equal.  (*i, *j) become the fluid cell;
 * *fx, *fy say which mirrors apply (each flips the moments mr_refl_flip
 * names for its axis). */
MR_INL void mr_step_mirror(const mr_inst& I, int* i, int* j, bool* fx, bool* fy) {
  const int dx = *i - I.stepi, dy = I.stepj - 1 - *j;
  *fx = dx <= dy;
  *fy = dy <= dx;
  if (*fx) *i = 2 * I.stepi - 1 - *i;
  if (*fy) *j = 2 * I.stepj - 1 - *j;
}

/* moment m of component c of the cell (i, j) of the extended grid if,
   after the domain's fold, it reads a cell of the step: the mirror image,
   loaded from the state U (planes of I.plane); false otherwise */
MR_INL bool mr_step_val(const mr_inst& I, const MR_GLB double* U, int c, int m, int i, int j, double* val) {
  if (I.stepj <= 0) return false;
  int kx = 0, ky = 0;
  int ii = mr_fold(i, I.nx, I.bcx, &kx), jj = mr_fold(j, I.ny, I.bcy, &ky);
  if (!mr_solid(I, ii, jj)) return false;
  bool sx, sy;
  mr_step_mirror(I, &ii, &jj, &sx, &sy);
  double v = U[(long long)(c * 3 + m) * I.plane + (long long)jj * I.nx + ii];
  v = ((((kx == 2) != sx) && mr_refl_flip(c, m, 0)) != (((ky == 2) != sy) && mr_refl_flip(c, m, 1))) ? -v : v;
  *val = ((kx == 1 || ky == 1) && m > 0) ? 0.0 : v;
  return true;
}

/* moment m of component c of a ghost cell with prescribed data (see
   mr_presc_any); false if the cell holds none */
MR_INL bool mr_presc(const mr_inst& I, int c, int m, int i, int j, double t, double* val) {
#pragma clang fp contract(off)
  if (I.dim == 2 && (j < 0 || j >= I.ny)) {
    const int s = j < 0 ? 2 : 3;
    if ((I.pres >> s) & 1) {
      const double xc = I.x0 + (i + 0.5) * I.dx, yc = I.y0 + (j + 0.5) * I.dy;
      const double A = I.spre[s][c];
      if (I.skind[s] == 3) {
        const double B = I.sstate[s][c];
        double a = 0.0, mx = 0.0, my = 0.0;
        if (I.ssplit[s][0] > -HUGE_VAL)
          mr_clip(I.dx, -I.ssplit[s][2] * I.dy, I.ssplit[s][0] + I.ssplit[s][1] * t + I.ssplit[s][2] * yc - xc,
                  &a, &mx, &my);
        *val = m == 0 ? B + (A - B) * a : (A - B) * (m == 1 ? mx : my);
        return true;
      }
      if (xc < I.ssplit[s][0] + I.ssplit[s][1] * t + I.ssplit[s][2] * yc) {
        *val = m == 0 ? A : 0.0;
        return true;
      }
    }
  }
  if (i < 0 || i >= I.nx) {
    const int s = i < 0 ? 0 : 1;
    if (((I.pres >> s) & 1) && I.skind[s] == 3) {
      *val = m == 0 ? I.sstate[s][c] : 0.0;
      return true;
    }
  }
  return false;
}

/* The x face f of row j (between cells (f-1, j) and (f, j)), or the y face
 * f of column i, is a reflective wall at time t: a face of the step --
 * continued through the ghost cells below the tunnel and beyond the exit,
 * where the ghost field is the mirror image across it as well -- or the
 * side is reflective and the ghost across the face holds no prescribed
 * state.  STEP = false: kernel variants for instances without a step. */
template <bool STEP = true>
MR_INL bool mr_wall_x(const mr_inst& I, int f, int j, double t) {
  if (STEP && I.stepj > 0 && f == I.stepi && j < I.stepj) return true;   /* the step's vertical face (and below) */
  if (!mr_wall(f, I.nx, I.bcx)) return false;
  return !((I.pres >> (f == 0 ? 0 : 1)) & 1) || !mr_presc_any(I, f == 0 ? -1 : I.nx, j, t);
}
template <bool STEP = true>
MR_INL bool mr_wall_y(const mr_inst& I, int i, int f, double t) {
  if (STEP && I.stepj > 0 && f == I.stepj && i >= I.stepi) return true;   /* the step's top (and beyond the exit) */
  if (!mr_wall(f, I.ny, I.bcy)) return false;
  return !((I.pres >> (f == 0 ? 2 : 3)) & 1) || !mr_presc_any(I, i, f == 0 ? -1 : I.ny, t);
}

struct mr_grid {
  const MR_GLB double* U;  /* state base: comp c, moment m plane at U + (c*nm + m)*P */
  long long P;
  int nx, ny, bcx, bcy, nm;
  const mr_inst* I;        /* instance with prescribed ghosts (or null), and
                              the time of its boundary data */
  double t;
};

/* moment m of component c at cell (i, j) with ghost handling: the folded
   cell is always loaded (it lies in the grid) and the ghost rules applied
   to the value, so that a run of these loads issues without branches; the
   prescribed data of an inflow side or front, rare, replace it last */
template <bool STEP = true>
MR_INL double mr_ld(const mr_grid& g, int c, int m, int i, int j) {
  int kx = 0, ky = 0;
  int ii = mr_fold(i, g.nx, g.bcx, &kx);
  int jj = (g.nm == 3) ? mr_fold(j, g.ny, g.bcy, &ky) : 0;
  bool sx = false, sy = false;   /* a cell of the step: its mirror image */
  if (STEP && g.I && g.I->stepj > 0 && mr_solid(*g.I, ii, jj)) mr_step_mirror(*g.I, &ii, &jj, &sx, &sy);
  double v = g.U[(long long)(c * g.nm + m) * g.P + (long long)jj * g.nx + ii];
  v = ((((kx == 2) != sx) && mr_refl_flip(c, m, 0)) != (((ky == 2) != sy) && mr_refl_flip(c, m, 1))) ? -v : v;
  v = ((kx == 1 || ky == 1) && m > 0) ? 0.0 : v;
  if (g.I && (kx | ky) && g.I->pres) {
    double pv;
    if (mr_presc(*g.I, c, m, i, j, g.t, &pv)) v = pv;
  }
  return v;
}

/* Step 1 of a 1D cell for its NC components from the three-cell stencil
 * (averages um, u0, up and first moments vm, v0, vp per component):
 * component by component, or, for Euler with I.charwise, on the
 * characteristic fields of the flux Jacobian at the cell's average u0 --
 * every stencil moment is projected with the left eigenvectors, each field
 * reconstructed, and the four values mapped back with the right ones.
 * Right eigenvectors (columns): (1, v-c, H-vc), (1, v, v^2/2), (1, v+c,
 * H+vc); left ones (rows) with b1 = (gamma-1)/c^2, b2 = b1 v^2/2:
 * ((b2 + v/c)/2, -(b1 v + 1/c)/2, b1/2), (1 - b2, b1 v, -b1),
 * ((b2 - v/c)/2, -(b1 v - 1/c)/2, b1/2). */
template <int NC, bool BP>
MR_INL void mr1_recon_sys(const double* um, const double* u0, const double* up, const double* vm,
                          const double* v0, const double* vp, const mr_inst& I, double (*out)[4]) {
  if (NC == 3 && I.charwise) {
    const double rho = u0[0], v = u0[1] / rho;
    const double p = (I.gam - 1.0) * (u0[2] - 0.5 * rho * v * v);
    const double c = sqrt(I.gam * p / rho), H = (u0[2] + p) / rho;
    const double b1 = (I.gam - 1.0) / (c * c), b2 = 0.5 * b1 * v * v;
    const double L[3][3] = {{0.5 * (b2 + v / c), -0.5 * (b1 * v + 1.0 / c), 0.5 * b1},
                            {1.0 - b2, b1 * v, -b1},
                            {0.5 * (b2 - v / c), -0.5 * (b1 * v - 1.0 / c), 0.5 * b1}};
    const double R[3][3] = {{1.0, 1.0, 1.0}, {v - c, v, v + c}, {H - v * c, 0.5 * v * v, H + v * c}};
    double w[3][4];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      auto pr = [&](const double* x) { return L[k][0] * x[0] + L[k][1] * x[1] + L[k][2] * x[2]; };
      mr_recon1d<BP>(pr(um), pr(u0), pr(up), pr(vm), pr(v0), pr(vp), I.W, w[k]);
    }
#pragma unroll
    for (int cc = 0; cc < 3; ++cc)
#pragma unroll
      for (int q = 0; q < 4; ++q) out[cc][q] = R[cc][0] * w[0][q] + R[cc][1] * w[1][q] + R[cc][2] * w[2][q];
    return;
  }
#pragma unroll
  for (int cc = 0; cc < NC; ++cc) mr_recon1d<BP>(um[cc], u0[cc], up[cc], vm[cc], v0[cc], vp[cc], I.W, out[cc]);
}

/* Characteristic-wise Step 1 in 2D (2D Euler, I.charwise): every cell
 * has one set of values per direction D (0: x, 1: y), reconstructed on the
 * characteristic fields of the flux Jacobian in direction D at the cell's
 * average.  With the normal velocity vn, the tangential velocity vt,
 * q^2 = u^2 + v^2, H = (E + p)/rho, b1 = (gamma-1)/c^2, b2 = b1 q^2/2, the
 * right eigenvectors (columns) are the acoustic waves (1, .., H -+ vn c)
 * with vn -+ c in the normal momentum slot, the entropy wave
 * (1, u, v, q^2/2) and the shear wave with a 1 in the tangential momentum
 * slot and vt in the energy slot; the left ones are their inverse's rows:
 * ((b2 + vn/c)/2, -(b1 vn + 1/c)/2, -b1 vt/2, b1/2), (1 - b2, b1 vn, b1 vt,
 * -b1), (-vt, 0, 1, 0), ((b2 - vn/c)/2, -(b1 vn - 1/c)/2, -b1 vt/2, b1/2),
 * entries listed in the order (rho, normal momentum, tangential momentum,
 * E).  Everything that belongs to direction D takes set D: the fluxes on
 * the faces normal to D, the volume integral of the flux in D, and in the
 * KXRCF test the jumps and the normal velocity on those faces; the KXRCF
 * norm is the maximum |rho| over both sets. */
struct mr_char2 {
  double vn, vt, c, rc, H, b1, b2, q2h;   /* q2h = q^2/2 */
};

template <int D>
MR_INL mr_char2 mr_char2_state(const double* u, double gam) {
  mr_char2 e;
  const double r = mr_rcp(u[0]);
  const double vx = u[1] * r, vy = u[2] * r;
  e.q2h = 0.5 * (vx * vx + vy * vy);
  const double p = (gam - 1.0) * (u[3] - u[0] * e.q2h);
  const double c2 = gam * p * r;
  e.c = mr_sqrtp(c2);
  e.rc = mr_rcp(e.c);
  e.H = (u[3] + p) * r;
  e.b1 = (gam - 1.0) * mr_rcp(c2);
  e.b2 = e.b1 * e.q2h;
  e.vn = D == 0 ? vx : vy;
  e.vt = D == 0 ? vy : vx;
  return e;
}

/* row k of L in conserved order (rho, rho u, rho v, E) */
template <int D>
MR_INL void mr_char2_left(const mr_char2& e, int k, double l[4]) {
  constexpr int N = 1 + D, T = 2 - D;
  double a0, an, at, ae;
  if (k == 0) { a0 = 0.5 * (e.b2 + e.vn * e.rc); an = -0.5 * (e.b1 * e.vn + e.rc); at = -0.5 * e.b1 * e.vt; ae = 0.5 * e.b1; }
  else if (k == 1) { a0 = 1.0 - e.b2; an = e.b1 * e.vn; at = e.b1 * e.vt; ae = -e.b1; }
  else if (k == 2) { a0 = -e.vt; an = 0.0; at = 1.0; ae = 0.0; }
  else { a0 = 0.5 * (e.b2 - e.vn * e.rc); an = -0.5 * (e.b1 * e.vn - e.rc); at = -0.5 * e.b1 * e.vt; ae = 0.5 * e.b1; }
  l[0] = a0; l[N] = an; l[T] = at; l[3] = ae;
}

/* conserved values from the four field values w (R w) */
template <int D>
MR_INL void mr_char2_right(const mr_char2& e, const double w[4], double out[4]) {
  constexpr int N = 1 + D, T = 2 - D;
  const double s = w[0] + w[1] + w[3];
  out[0] = s;
  out[N] = e.vn * s + e.c * (w[3] - w[0]);
  out[T] = e.vt * s + w[2];
  out[3] = e.H * (w[0] + w[3]) + e.vn * e.c * (w[3] - w[0]) + e.q2h * w[1] + e.vt * w[2];
}

/* flag of cell (i, j) from an extended plane with halo h (clamped) */
template <class P>
MR_INL int mr_flag(P fl, int ex, int ey, int h, int i, int j) {
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
MR_INL void mr2_cell_values(const mr_grid& g, const mr_inst& I, const MR_GLB unsigned char* fl,
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

/* Final Gauss-Lobatto values of all four components of cell (x, y), set D
 * of the characteristic-wise Step 1 (see mr_char2): each field is
 * projected from the stencil (with the troubled cells' first moments
 * modified if the cell is troubled), reconstructed, and mapped back. */
template <bool BP, int D>
MR_INL void mr2_cell_values_ch(const mr_grid& g, const mr_inst& I, const MR_GLB unsigned char* fl, int x, int y,
                               double out[4][16]) {
  int fs[9];
#pragma unroll
  for (int l = 0; l < 9; ++l) fs[l] = mr_flag(fl, I.fex, I.fey, I.fhalo, x + l % 3 - 1, y + l / 3 - 1);
  double u0[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) u0[c] = mr_ld(g, c, 0, x, y);
  const mr_char2 e = mr_char2_state<D>(u0, I.gam);
#pragma unroll
  for (int c = 0; c < 4; ++c)
#pragma unroll
    for (int q = 0; q < 16; ++q) out[c][q] = 0.0;
  double w[4][16];
#pragma unroll 1
  for (int k = 0; k < 4; ++k) {
    double lk[4];
    mr_char2_left<D>(e, k, lk);
    double fu[9], fv[9], fw[9];
    for (int l = 0; l < 9; ++l) { fu[l] = 0.0; fv[l] = 0.0; fw[l] = 0.0; }
    for (int c = 0; c < 4; ++c) {
      double u[9], v[9], ww[9];
      for (int l = 0; l < 9; ++l) {
        u[l] = mr_ld(g, c, 0, x + l % 3 - 1, y + l / 3 - 1);
        v[l] = mr_ld(g, c, 1, x + l % 3 - 1, y + l / 3 - 1);
        ww[l] = mr_ld(g, c, 2, x + l % 3 - 1, y + l / 3 - 1);
      }
      if (fs[4]) mr2_modify_stencil(g, c, x, y, fs, v, ww);
      for (int l = 0; l < 9; ++l) { fu[l] += lk[c] * u[l]; fv[l] += lk[c] * v[l]; fw[l] += lk[c] * ww[l]; }
    }
    mr_recon2d<BP>(fu, fv, fw, I.W, w[k]);
  }
  for (int q = 0; q < 16; ++q) {
    const double wq[4] = {w[0][q], w[1][q], w[2][q], w[3][q]};
    double o[4];
    mr_char2_right<D>(e, wq, o);
    for (int c = 0; c < 4; ++c) out[c][q] = o[c];
  }
}

/* KXRCF face data of cell (i, j) from its Step-1 values, eqs. (KXRCF_),
 * (line-integral-average_): f[0..3] Gauss-Lobatto means of the indicator
 * variable (density; u for Burgers) on the left, right, bottom, top face,
 * f[4..7] the same for the normal velocity, f[8] the max |u| over the 16
 * points. */
template <bool BP>
MR_INL void mr2_face_summary(const mr_grid& g, const mr_inst& I, int i, int j, double f[9]) {
  double irl[4], irr[4], irm[4];   /* 1/rho at points 0,4,8,12 | 3,7,11,15 | 1,2,13,14 */
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
    mr_recon2d<BP>(u, v, w, I.W, r);
    if (c == 0) {
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        sl += glw(m) * r[0 + 4 * m];
        sr += glw(m) * r[3 + 4 * m];
        sb += glw(m) * r[m];
        st += glw(m) * r[12 + m];
      }
#pragma unroll
      for (int k = 0; k < 16; ++k) nrm = fmax(nrm, fabs(r[k]));
      if (ncomp == 1) { vl = sl; vr = sr; vb = sb; vt = st; }   /* Burgers: f'(u) = u */
      else {
        mr_recip4(r[0], r[4], r[8], r[12], irl);
        mr_recip4(r[3], r[7], r[11], r[15], irr);
        mr_recip4(r[1], r[2], r[13], r[14], irm);
      }
    } else if (c == 1) {
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        vl += glw(m) * (r[0 + 4 * m] * irl[m]);
        vr += glw(m) * (r[3 + 4 * m] * irr[m]);
      }
    } else {
      vb = glw(0) * (r[0] * irl[0]) + glw(1) * (r[1] * irm[0]) + glw(2) * (r[2] * irm[1]) + glw(3) * (r[3] * irr[0]);
      vt = glw(0) * (r[12] * irl[3]) + glw(1) * (r[13] * irm[2]) + glw(2) * (r[14] * irm[3]) + glw(3) * (r[15] * irr[3]);
    }
  }
  f[0] = sl; f[1] = sr; f[2] = sb; f[3] = st;
  f[4] = vl; f[5] = vr; f[6] = vb; f[7] = vt;
  f[8] = nrm;
}

template <int NC, int D>
MR_INL void mr_numflux(const double* a, const double* b, double gam, double alpha, double* f) {
  if constexpr (NC == 1) f[0] = mr_lf(a[0], b[0], alpha);
  else mr_hllc<NC, D>(a, b, gam, f);
}

/* Flux through a wall face normal to direction D of the fluid trace u,
 * the wall on side sgn (+1: towards +D): the Godunov flux of the
 * mirror-image Riemann problem, whose star state is at rest -- mass and
 * energy flux zero, normal momentum flux the star pressure p*.  With u_n
 * the velocity into the wall, p* solves the shock relation
 * (p* - p) sqrt(A / (p* + B)) = u_n (A = 2/((g+1) rho), B = (g-1)/(g+1) p)
 * for u_n > 0, taken as the positive root q = p* - p of
 * A q^2 - u_n^2 q - u_n^2 (p + B) = 0; the isentropic rarefaction
 * p* = p (1 + (g-1) u_n/(2c))^(2g/(g-1)) for u_n < 0 (0 at vacuum);
 * p* = p for u_n = 0. */
template <int D>
MR_INL void mr_wall_flux(const double* u, int sgn, double gam, double* f) {
  const double p = mr_pressure<4>(u, gam);
  const double un = sgn * (u[1 + D] / u[0]);
  double ps = p;
  if (un > 0.0) {
    const double A = 2.0 / ((gam + 1.0) * u[0]), B = (gam - 1.0) / (gam + 1.0) * p;
    ps = p + un * (un + sqrt(un * un + 4.0 * A * (p + B))) / (2.0 * A);
  } else if (un < 0.0) {
    const double c = sqrt(gam * p / u[0]);
    const double base = 1.0 + 0.5 * (gam - 1.0) * un / c;
    ps = base > 0.0 ? p * pow(base, 2.0 * gam / (gam - 1.0)) : 0.0;
  }
  f[0] = 0.0;
  f[1] = 0.0;
  f[2] = 0.0;
  f[3] = 0.0;
  f[1 + D] = ps;
}

/* numerical flux at a point of face f (D = 0: the x face f of row `other`;
 * D = 1: the y face f of column `other`) from the traces a (low side) and
 * b (high side): on a wall face of an instance with wallflux set, the wall
 * flux of the fluid trace -- the fluid lies on the low side of the
 * domain's high walls and of the step's vertical face, on the high side of
 * the low walls and of the step's top -- else mr_numflux */
template <int NC, int D, bool GB>
MR_INL void mr_face_flux(const mr_inst& I, const double* a, const double* b, double gam, double alpha, int f,
                         int other, double tb, double* out) {
  if constexpr (GB && NC == 4) {
    if (I.wallflux && (D == 0 ? mr_wall_x(I, f, other, tb) : mr_wall_y(I, other, f, tb))) {
      const bool low = D == 0 ? f != 0 : f == I.ny;
      mr_wall_flux<D>(low ? a : b, low ? 1 : -1, gam, out);
      return;
    }
  }
  mr_numflux<NC, D>(a, b, gam, alpha, out);
}

template <int NC, int D>
MR_INL void mr_physflux(const double* u, double gam, double* f) {
  if constexpr (NC == 1) f[0] = 0.5 * u[0] * u[0];
  else mr_euler_flux<NC, D>(u, gam, f);
}

/* exchange with lane ^ 1 or lane ^ 2 inside a group of four lanes, through
 * the DPP quad permutation (no LDS traffic) */
template <int X>
MR_INL double mr_quad_xor(double v) {
  constexpr int ctrl = X == 1 ? 0xB1 : 0x4E;   /* quad_perm [1,0,3,2] / [2,3,0,1] */
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffffll), ctrl, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), ctrl, 0xF, 0xF, true);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (long long)(unsigned)lo);
}

/* reduce-scatter over the NC lanes of a cell: lane k receives sum_r a_r[k] */
template <int NC>
MR_INL double mr_rs(const double (&a)[NC], int k) {
  if (NC == 1) return a[0];
  const bool hi = (k & 2) != 0;
  const double s0 = hi ? a[0] : a[2], s1 = hi ? a[1] : a[3];
  const double k0 = hi ? a[2] : a[0], k1 = hi ? a[3] : a[1];
  const double b0 = k0 + mr_quad_xor<2>(s0);
  const double b1 = k1 + mr_quad_xor<2>(s1);
  const bool odd = (k & 1) != 0;
  const double s = odd ? b0 : b1, kk = odd ? b1 : b0;
  return kk + mr_quad_xor<1>(s);
}

/* 2D final Gauss-Lobatto values of interior cells: gl[(c*16 + p)*plane + cell]. */
