/* Host side of the MR-HWENO C ABI (include/mrhweno.h): validation,
 * workspace layout, work lists, hipGraph capture of one SSP-RK3 step,
 * state hand-back and the one-off probes (reconstruct / flag / residual). */
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstddef>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/mrhweno.h"
#include "mr_mlp.h"
#include "mr_types.h"

extern "C" {
hipError_t mr_launch_reduce(hipStream_t, mr_inst*, const mr_tile1*, int, int);
hipError_t mr_launch_finalize(hipStream_t, mr_inst*, int, int);
hipError_t mr_launch_summary(hipStream_t, int, int, int, mr_inst*, const mr_tile1*, int, int);
hipError_t mr_launch_flags(hipStream_t, int, mr_inst*, const mr_tile1*, int, int);
hipError_t mr_launch_stage1(hipStream_t, int, int, int, mr_inst*, const mr_tile1*, int, int, int);
hipError_t mr_launch_fused1(hipStream_t, int, int, int, mr_inst*, const mr_tile1*, int, int);
hipError_t mr_launch_stage2(hipStream_t, int, int, int, int, mr_inst*, const mr_tile2*, int, int, int);
hipError_t mr_launch_kxrcf2(hipStream_t, int, int, int, mr_inst*, const mr_tile2*, int, int);
hipError_t mr_launch_values(hipStream_t, int, int, int, mr_inst*, const mr_tile1*, int, double*);
hipError_t mr_launch_fb_reset(hipStream_t, int*, int);
hipError_t mr_launch_pack(hipStream_t, const void*, mr_learn_w*);
hipError_t mr_launch_learned(hipStream_t, mr_inst*, const mr_tile2*, int, int, const mr_learn_w*, mr_band*, int*, int);
hipError_t mr_launch_fallback(hipStream_t, mr_inst*, const mr_band*, int*, int, int, int);
hipError_t mr_launch_features(hipStream_t, const mr_inst*, int, const int*, int, void*);
size_t mr_mlp_cache_bytes(int);
hipError_t mr_mlp_gemm(hipStream_t, int, int, int, const void*, long long, long long, const void*, long long,
                       long long, void*, long long, long long);
hipError_t mr_mlp_forward(hipStream_t, const void*, const void*, void*, void*, int);
hipError_t mr_mlp_backward(hipStream_t, const void*, const void*, void*, const void*, void*, void*, int);
hipError_t mr_mlp_adam(hipStream_t, void*, void*, const void*, void*, void*, int, float, float, float, float);
}

namespace {

constexpr int kBlock = 256;
constexpr int kFused1 = kBlock - 6;   /* cells of a tile of the step's 1D kernel (three ring cells each side) */
constexpr int kFHalo = 2;   /* flags: final values of cells -1..n need flags -2..n+1 */
constexpr int kSHalo = 3;   /* summaries: flags of cells -2..n+1 need summaries -3..n+2 */
constexpr int kMinRows = 8; /* smallest 2D strip height the work lists are sized for */
constexpr int kKxW = 62;    /* 2D KXRCF work item: 62 flag columns ...                */
constexpr int kKxRows = 46; /* ... x up to 46 flag rows of the extended flag range    */
constexpr int kKxMinRows = 8;
constexpr int kKxMaxRows = 256; /* tallest height a caller may set */
constexpr int kKxFill = 512; /* work groups that fill the GPU (256 CUs x 2 resident)    */
constexpr int kLearnW = 64;     /* learned-indicator work item: 64 columns ...       */
constexpr int kLearnRows = 32;  /* ... x 32 rows of the extended flag range          */

thread_local std::string g_err;

size_t al(size_t x) { return (x + 255) & ~size_t(255); }

int ncomp_of(const mrhweno_problem& p) { return p.flux == MRHWENO_BURGERS_LF ? 1 : (p.dim == 1 ? 3 : 4); }
long long plane_of(const mrhweno_problem& p) { return (long long)p.nx * (p.dim == 2 ? p.ny : 1); }
size_t state_bytes(const mrhweno_problem& p) { return sizeof(double) * ncomp_of(p) * (p.dim + 1) * plane_of(p); }
int ext(int n, int h) { return n + 2 * h; }
int ceil_div_i(int a, int b) { return (a + b - 1) / b; }
int fex(const mrhweno_problem& p) { return ext(p.nx, kFHalo); }
int fey(const mrhweno_problem& p) { return p.dim == 2 ? ext(p.ny, kFHalo) : 1; }
int sex(const mrhweno_problem& p) { return ext(p.nx, kSHalo); }
int sey(const mrhweno_problem& p) { return p.dim == 2 ? ext(p.ny, kSHalo) : 1; }
int nsumm(const mrhweno_problem& p) { return p.dim == 1 ? 5 : 9; }
bool learned(const mrhweno_problem& p) { return p.tc_mode == MRHWENO_TC_LEARNED; }
bool kxrcf(const mrhweno_problem& p) { return p.tc_mode == MRHWENO_TC_KXRCF; }
bool tvb(const mrhweno_problem& p) { return p.tc_mode == MRHWENO_TC_TVB; }
/* an indicator pass of its own (KXRCF or TVB; the learned one has its kernel) */
bool indicator_pass(const mrhweno_problem& p) { return kxrcf(p) || tvb(p); }
/* 1D KXRCF keeps face summaries in a plane; 2D KXRCF computes them in LDS */
bool needs_summ(const mrhweno_problem& p) { return indicator_pass(p) && p.dim == 1; }
/* side s (0 left, 1 right, 2 bottom, 3 top) carries boundary data: an
   inflow state or a front */
bool side_data(const mrhweno_problem& p, int s) {
  const int bc = s < 2 ? p.bc_x : p.bc_y;
  return bc == MRHWENO_BC_SIDES && (p.side[s].kind == MRHWENO_SIDE_INFLOW || p.side[s].front);
}
/* work items of the learned indicator: strips over [-2, n+2)^2 */
int learn_tiles(const mrhweno_problem& p) {
  return learned(p) ? ceil_div_i(ext(p.nx, kFHalo), kLearnW) * ceil_div_i(ext(p.ny, kFHalo), kLearnRows) : 0;
}
int strip_cells(const mrhweno_problem& p) { return kBlock / ncomp_of(p); }   /* 2D strip width incl. ring */
/* rows of a 2D KXRCF work item: 46 (each strip also reconstructs a ring row
   above and below), fewer for grids too small to fill the GPU otherwise */
int kx_rows(const mrhweno_problem& p) {
  /* the height that minimises waves of kKxFill resident work groups times
     the sweep steps (four rows each) of a strip; the tallest among equals.
     A small last wave would double the kernel's time. */
  const int cols = ceil_div_i(ext(p.nx, kFHalo), kKxW), ey = ext(p.ny, kFHalo);
  int best = kKxMinRows;
  long long bc = -1;
  for (int r = kKxMinRows; r <= kKxRows; ++r) {
    const long long tiles = (long long)cols * ceil_div_i(ey, r);
    const long long cost = ((tiles + kKxFill - 1) / kKxFill) * ceil_div_i(r + 2, 4);
    if (bc < 0 || cost <= bc) { bc = cost; best = r; }
  }
  return best;
}
/* 2D KXRCF work items: strips over [-2, n+2)^2, `rows` rows each (0: the
   height of kx_rows) */
int kx_tiles(const mrhweno_problem& p, int rows = 0) {
  return p.dim == 2 && indicator_pass(p)
             ? ceil_div_i(ext(p.nx, kFHalo), kKxW) * ceil_div_i(ext(p.ny, kFHalo), rows > 0 ? rows : kx_rows(p))
             : 0;
}

std::string validate(const mrhweno_problem& p) {
  if (p.dim != 1 && p.dim != 2) return "dim must be 1 or 2";
  if (p.nx < 8 || (p.dim == 2 && p.ny < 8)) return "grid must have at least 8 cells per direction";
  if (!(p.x1 > p.x0) || (p.dim == 2 && !(p.y1 > p.y0))) return "empty domain";
  if (p.flux != MRHWENO_BURGERS_LF && p.flux != MRHWENO_EULER_HLLC) return "unknown flux";
  if (p.bc_x < 0 || p.bc_x > 3 || (p.dim == 2 && (p.bc_y < 0 || p.bc_y > 3))) return "unknown boundary condition";
  for (int s = 0; s < (p.dim == 2 ? 4 : 2); ++s) {
    const int bc = s < 2 ? p.bc_x : p.bc_y;
    const int kind = bc == MRHWENO_BC_SIDES ? p.side[s].kind : bc;
    if (kind == MRHWENO_BC_REFLECTIVE && p.flux != MRHWENO_EULER_HLLC) return "reflective walls are for the Euler equations";
    if (bc != MRHWENO_BC_SIDES) continue;
    const mrhweno_side& sd = p.side[s];
    if (sd.kind < MRHWENO_SIDE_TRANSMISSIVE || sd.kind > MRHWENO_SIDE_INFLOW) return "unknown side kind";
    if (sd.front != 0 && sd.front != 1) return "side front must be 0 or 1";
    if (sd.front && s < 2) return "a front is defined on the bottom and top sides only";
    for (int q = 0; q < 3; ++q)
      if (sd.front && !std::isfinite(sd.split[q])) return "side front coefficients must be finite";
    for (int w = 0; w < 2; ++w) {
      if (w == 0 ? sd.kind != MRHWENO_SIDE_INFLOW : !sd.front) continue;
      const double* u = w == 0 ? sd.state : sd.pre;
      for (int c = 0; c < ncomp_of(p); ++c)
        if (!std::isfinite(u[c])) return "prescribed side states must be finite";
      if (p.flux == MRHWENO_EULER_HLLC) {
        const int nc = ncomp_of(p);
        double ke = 0.0;
        for (int c = 1; c < nc - 1; ++c) ke += 0.5 * u[c] * u[c] / u[0];
        if (!(u[0] > 0.0) || !(u[nc - 1] - ke > 0.0)) return "prescribed side states must have positive density and pressure";
      }
    }
  }
  if (p.tc_mode == MRHWENO_TC_LEARNED && (p.bc_x == MRHWENO_BC_SIDES || p.bc_y == MRHWENO_BC_SIDES))
    return "the learned indicator takes no per-side boundary data";
  if (p.flux == MRHWENO_EULER_HLLC && !(p.gamma_gas > 1.0)) return "gamma_gas must exceed 1";
  if (!(p.cfl > 0.0) || !(p.t_final > 0.0)) return "cfl and t_final must be positive";
  for (int l = 0; l < 4; ++l)
    if (!(p.gamma_bar[l] > 0.0) || !std::isfinite(p.gamma_bar[l])) return "linear weights must be positive";
  if (!(p.eps > 0.0)) return "eps must be positive";
  if (p.tc_mode < 0 || p.tc_mode > 4) return "unknown troubled-cell mode";
  if (!(p.tvb_m >= 0.0) || !std::isfinite(p.tvb_m)) return "tvb_m must be finite and non-negative";
  if (p.beta_on != 0 && p.beta_on != 1) return "unknown beta_on";
  if (p.modification < 0 || p.modification > 2) return "unknown modification placement";
  if (p.charwise != 0 && p.charwise != 1) return "charwise must be 0 or 1";
  if (p.charwise && p.flux != MRHWENO_EULER_HLLC) return "characteristic-wise reconstruction is for the Euler equations";
  if (p.charwise && p.dim == 2 && (p.tc_mode == MRHWENO_TC_LEARNED || p.tc_mode == MRHWENO_TC_TVB))
    return "2D characteristic-wise reconstruction takes the KXRCF, all-cells or no troubled-cell mode";
  if (p.tc_mode == MRHWENO_TC_LEARNED && (p.dim != 2 || p.flux != MRHWENO_EULER_HLLC))
    return "the learned indicator is for 2D Euler";
  if (p.dim == 2) {
    const double dx = (p.x1 - p.x0) / p.nx, dy = (p.y1 - p.y0) / p.ny;
    if (std::fabs(dx - dy) > 1e-12 * std::max(dx, dy)) return "2D cells must be square (dx == dy)";
  }
  if (p.wall_flux != 0 && p.wall_flux != 1) return "wall_flux must be 0 or 1";
  if (p.wall_flux && (p.dim != 2 || p.flux != MRHWENO_EULER_HLLC)) return "wall_flux is for 2D Euler";
  if (p.step_j != 0) {
    if (p.dim != 2 || p.flux != MRHWENO_EULER_HLLC) return "a step is for 2D Euler";
    if (p.step_j < 0 || p.step_i < 1 || p.step_i >= p.nx || p.step_j > p.step_i || 2 * p.step_j > p.ny)
      return "the step needs 0 < step_j <= step_i < nx and 2 step_j <= ny (its mirror images lie in the grid)";
    if (p.tc_mode != MRHWENO_TC_NONE && p.tc_mode != MRHWENO_TC_KXRCF && p.tc_mode != MRHWENO_TC_ALL)
      return "a step takes the KXRCF, all-cells or no troubled-cell mode";
  }
  /* 1D: cell, summary and flag indices (the grid plus its halos, a block
     of threads past the last cell) stay in 32 bits */
  if (p.dim == 1 && p.nx >= (1 << 30)) return "1D grid too large (at most 2^30 - 1 cells)";
  if (plane_of(p) > (1ll << 31) - 1) return "grid too large";
  /* the 2D stage kernel addresses a moment plane and row as a 30-bit offset */
  if (p.dim == 2 && 13ll * plane_of(p) >= (1ll << 30)) return "2D grid too large (at most 2^30/13 cells)";
  return "";
}

/* workspace layout, computed identically for sizing and for creation */
struct Layout {
  size_t insts = 0, tiles1 = 0, tiles2 = 0, probe_tiles = 0, probe_aleph = 0, total = 0;
  size_t lw = 0, cnt = 0, band = 0, tilesl = 0;   /* learned indicator */
  std::vector<size_t> buf1, buf2, unm, fl0, fl1, summ;
  size_t n_tiles1 = 0, n_tiles2 = 0, n_probe_tiles = 0, n_tilesl = 0, n_band = 0;
};

int ceil_div(long long a, long long b) { return (int)((a + b - 1) / b); }

Layout layout(const mrhweno_problem* P, int n) {
  Layout L;
  size_t off = 0;
  L.insts = off;
  off += al(sizeof(mr_inst) * (n + 1));
  /* per-cell work items: reduce (plane), summary (extended), flags (extended),
     values (plane), 1D stage (block tiles) */
  size_t t1 = 0, t2 = 0, tmax = 0;
  for (int q = 0; q < n; ++q) {
    const auto& p = P[q];
    size_t a = ceil_div(plane_of(p), kBlock) + ceil_div((long long)sex(p) * sey(p), kBlock) +
               ceil_div((long long)fex(p) * fey(p), kBlock) + ceil_div(plane_of(p), kBlock);
    if (p.dim == 1) a += ceil_div(p.nx, kFused1);
    else t2 += (size_t)ceil_div(p.nx, strip_cells(p) - 2) * ceil_div(p.ny, kMinRows) + kx_tiles(p, kKxMinRows);
    t1 += a;
    tmax = std::max(tmax, a + learn_tiles(p) + kx_tiles(p) +
                              (p.dim == 2 ? (size_t)ceil_div(p.nx, strip_cells(p) - 2) * ceil_div(p.ny, kMinRows) : 0));
    L.n_tilesl += learn_tiles(p);
    if (learned(p)) L.n_band += (size_t)fex(p) * fey(p);
  }
  L.n_tiles1 = t1;
  L.n_tiles2 = t2;
  L.n_probe_tiles = tmax;
  L.tiles1 = off;
  off += al(sizeof(mr_tile1) * std::max<size_t>(t1, 1));
  L.tiles2 = off;
  off += al(sizeof(mr_tile2) * std::max<size_t>(t2, 1));
  L.probe_tiles = off;
  off += al(sizeof(mr_tile2) * (tmax + 64));
  if (L.n_tilesl) {
    L.lw = off; off += al(sizeof(mr_learn_w));
    L.cnt = off; off += al(16 * sizeof(int));
    L.band = off; off += al(sizeof(mr_band) * L.n_band);
    L.tilesl = off; off += al(sizeof(mr_tile2) * L.n_tilesl);
  }
  long long maxplane = 1;
  for (int q = 0; q < n; ++q) maxplane = std::max(maxplane, plane_of(P[q]));
  L.probe_aleph = off;
  off += al(sizeof(double) * 2 * maxplane);
  for (int q = 0; q < n; ++q) {
    const auto& p = P[q];
    L.buf1.push_back(off); off += al(state_bytes(p));
    L.buf2.push_back(off); off += al(state_bytes(p));
    L.unm.push_back(off);
    if (p.dim == 2) off += al(sizeof(double) * ncomp_of(p) * 2 * (size_t)plane_of(p));
    L.fl0.push_back(off); off += al((size_t)fex(p) * fey(p));
    L.fl1.push_back(off); off += al((size_t)fex(p) * fey(p));
    L.summ.push_back(off);
    if (needs_summ(p)) off += al(sizeof(double) * nsumm(p) * (size_t)sex(p) * sey(p));
  }
  L.total = off;
  return L;
}

/* host-side description of one launch group (instances sharing a kernel) */
struct Group {
  int dim, nc, bp;
  int gb;           /* boundary-data kernel variant (gb_of) */
  int ch;           /* 2D characteristic-wise Step 1 */
  bool any_summ = false, any_lf = false;
  std::vector<int> insts;
  int t_summ = 0, n_summ = 0, t_flag = 0, n_flag = 0, t_st1 = 0, n_st1 = 0;
  int t_st2 = 0, n_st2 = 0, t_kx = 0, n_kx = 0, t_tvb = 0, n_tvb = 0;
};

/* learned-indicator work items of one instance (instance id `slot`) */
void add_kx_tiles(std::vector<mr_tile2>& v, int slot, const mrhweno_problem& p, int rows_set = 0) {
  const int rows = rows_set > 0 ? rows_set : kx_rows(p);
  for (int y0 = -kFHalo; y0 < p.ny + kFHalo; y0 += rows)
    for (int x0 = -kFHalo; x0 < p.nx + kFHalo; x0 += kKxW)
      v.push_back(mr_tile2{slot, x0, y0, std::min(rows, p.ny + kFHalo - y0)});
}

/* XCD-aware order of the work items v[begin, end) of one instance.  The
   hardware hands work group i of a launch to XCD i % nxcd (round robin over
   the XCDs, each with its own L2), and a work group of a persistent grid
   whose size is a multiple of nxcd keeps that XCD for its later items.  The
   instance's natural order (row of strips after row of strips) is cut into
   nxcd contiguous runs of equal length, run j going to the slots
   begin + i nxcd + j, so the strips one XCD works on at a time are
   neighbours and their shared halo columns are read into the same L2.  It
   is done per instance: the items of one instance cost about the same, so
   every XCD gets an equal share, and the order of the instances in a batch
   (largest first, for a short tail) stays.  Results do not depend on the
   order. */
void xcd_order(std::vector<mr_tile2>& v, size_t begin, int nxcd) {
  const size_t n = v.size() - begin;
  if (nxcd <= 1 || n <= (size_t)nxcd) return;
  std::vector<mr_tile2> nat(v.begin() + begin, v.end());
  const size_t base = n / nxcd, extra = n % nxcd;   /* runs 0..extra-1 hold one more */
  size_t start = 0;
  for (int j = 0; j < nxcd; ++j) {
    const size_t len = base + ((size_t)j < extra ? 1 : 0);
    for (size_t i = 0; i < len; ++i) v[begin + i * nxcd + j] = nat[start + i];
    start += len;
  }
}

void add_learn_tiles(std::vector<mr_tile2>& v, int slot, const mrhweno_problem& p) {
  for (int y0 = -kFHalo; y0 < p.ny + kFHalo; y0 += kLearnRows)
    for (int x0 = -kFHalo; x0 < p.nx + kFHalo; x0 += kLearnW)
      v.push_back(mr_tile2{slot, x0, y0, std::min(kLearnRows, p.ny + kFHalo - y0)});
}

}  // namespace

struct mrhweno_ctx {
  int n = 0;
  hipStream_t stream = nullptr;
  char* ws = nullptr;
  Layout L;
  std::vector<mrhweno_problem> probs;
  std::vector<mr_inst> h;       /* host mirror of the descriptors */
  mr_inst* d = nullptr;
  mr_tile1* t1 = nullptr;
  mr_tile2* t2 = nullptr;
  int t_reduce = 0, n_reduce = 0;
  std::vector<Group> groups;
  std::vector<mr_tile1> h_t1;
  std::vector<mr_tile2> h_t2;
  int rows2 = 32, grid2 = 0;
  int kx_rows2 = 0;   /* rows of a 2D KXRCF work item (0: chosen per problem) */
  int nxcd = 1;       /* XCDs of the device (work-list order) */
  /* learned indicator */
  bool any_learned = false, weights_set = false;
  mr_learn_w* lw = nullptr;
  int* cnt = nullptr;
  mr_band* band = nullptr;
  mr_tile2* tl = nullptr;
  int n_tl = 0, grid_l = 512, grid_fb = 1024;
  int learned_bp = 0;   /* some learned instance takes beta on p_l */
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  bool any_lf = false;
  std::string err;
};

static mrhweno_status fail(mrhweno_ctx* c, mrhweno_status s, const std::string& m) {
  g_err = m;
  if (c) c->err = m;
  return s;
}

#define MR_CHECK(ctx, expr)                                                           \
  do {                                                                                \
    hipError_t e_ = (expr);                                                           \
    if (e_ != hipSuccess)                                                             \
      return fail(ctx, MRHWENO_ERR_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

static void fill_wconst(const mrhweno_problem& p, mr_wconst& W) {
  double S[4];
  double s = 0.0;
  for (int l = 0; l < 4; ++l) { s += p.gamma_bar[l]; S[l] = s; }
  for (int l = 0; l < 4; ++l) W.g4[l] = p.gamma_bar[l] / S[3];
  for (int l = 0; l < 4; ++l) W.sg[l] = S[l] / p.gamma_bar[l];
  for (int l = 0; l < 3; ++l) W.sgn[l] = S[l] / p.gamma_bar[l + 1];
  W.eps = p.eps;
}

/* the static part of an instance descriptor (grid, boundary data, flux,
   variants, weights); buffers and the dynamic part are left zero */
/* kernel variant for the instance's boundary data: 0 none, 1 ghosts that
   hold a prescribed state, 2 also a step or the wall flux */
static int gb_of(const mr_inst& I) { return (I.stepj > 0 || I.wallflux != 0) ? 2 : (I.pres != 0 ? 1 : 0); }

static void fill_inst(const mrhweno_problem& p, mr_inst& I) {
  std::memset(&I, 0, sizeof I);
  I.dim = p.dim; I.nx = p.nx; I.ny = p.dim == 2 ? p.ny : 1; I.nc = ncomp_of(p);
  I.flux = p.flux;
  I.x0 = p.x0; I.y0 = p.dim == 2 ? p.y0 : 0.0;
  /* fold kinds per side (low side in bits 0-1, high side in bits 2-3; an
     inflow side folds as a transmissive one and its ghosts are then
     overwritten) and the prescribed-ghost data */
  int fold[4] = {0, 0, 0, 0};
  for (int s = 0; s < (p.dim == 2 ? 4 : 2); ++s) {
    const int bc = s < 2 ? p.bc_x : p.bc_y;
    const int kind = bc == MRHWENO_BC_SIDES ? p.side[s].kind : bc;
    fold[s] = kind == MRHWENO_SIDE_INFLOW ? 1 : kind;
    I.skind[s] = kind;
    I.ssplit[s][0] = -HUGE_VAL;
    if (bc != MRHWENO_BC_SIDES) continue;
    const mrhweno_side& sd = p.side[s];
    for (int c = 0; c < 4; ++c) { I.sstate[s][c] = sd.state[c]; I.spre[s][c] = sd.pre[c]; }
    if (sd.front)
      for (int q = 0; q < 3; ++q) I.ssplit[s][q] = sd.split[q];
    if (sd.kind == MRHWENO_SIDE_INFLOW || sd.front) I.pres |= 1 << s;
  }
  I.bcx = fold[0] | (fold[1] << 2);
  I.bcy = fold[2] | (fold[3] << 2);
  I.stepi = p.dim == 2 && p.step_j > 0 ? p.step_i : 0;
  I.stepj = p.dim == 2 ? p.step_j : 0;
  I.wallflux = p.wall_flux;
  I.tc = p.tc_mode; I.beta_on = p.beta_on; I.mod = p.modification; I.charwise = p.charwise;
  I.fhalo = kFHalo; I.shalo = kSHalo;
  I.fex = fex(p); I.fey = fey(p); I.sex = sex(p); I.sey = sey(p);
  I.plane = plane_of(p);
  I.dx = (p.x1 - p.x0) / p.nx;
  I.dy = p.dim == 2 ? (p.y1 - p.y0) / p.ny : 1.0;
  I.gam = p.gamma_gas; I.cfl = p.cfl; I.t_final = p.t_final;
  I.rdx = 1.0 / I.dx;
  I.rdy = 1.0 / I.dy;
  I.band_lo = 0.2; I.band_hi = 0.8;
  I.tvb_mh2 = p.tvb_m * I.dx * I.dx;
  fill_wconst(p, I.W);
}

/* per-cell work items over `count` cells starting at 0 */
static void add_cells(std::vector<mr_tile1>& v, int inst, long long count) {
  for (long long s = 0; s < count; s += kBlock)
    v.push_back(mr_tile1{inst, (int)s, (int)std::min<long long>(kBlock, count - s), 0});
}

static void add_kx_tiles_if(std::vector<mr_tile2>& v, int q, const mrhweno_problem& p, bool want_tvb, int rows,
                            int nxcd) {
  if (kx_tiles(p) > 0 && tvb(p) == want_tvb) {
    const size_t first = v.size();
    add_kx_tiles(v, q, p, rows);
    xcd_order(v, first, nxcd);
  }
}

static void build_lists(mrhweno_ctx* c) {
  c->h_t1.clear();
  c->h_t2.clear();
  const int n = c->n;
  c->t_reduce = 0;
  for (int q = 0; q < n; ++q) add_cells(c->h_t1, q, plane_of(c->probs[q]));
  c->n_reduce = (int)c->h_t1.size();
  for (auto& g : c->groups) {
    g.t_summ = (int)c->h_t1.size();
    for (int q : g.insts)   /* 1D Step 2.1 runs inside the step's stage kernel (k1_fused) */
      if (g.dim == 2 && needs_summ(c->probs[q])) add_cells(c->h_t1, q, (long long)sex(c->probs[q]) * sey(c->probs[q]));
    g.n_summ = (int)c->h_t1.size() - g.t_summ;
    g.t_flag = (int)c->h_t1.size();
    for (int q : g.insts)   /* 2D KXRCF and TVB flags come from the fused kernel */
      if (g.dim == 2 && !learned(c->probs[q]) && !indicator_pass(c->probs[q]))
        add_cells(c->h_t1, q, (long long)fex(c->probs[q]) * fey(c->probs[q]));
    g.n_flag = (int)c->h_t1.size() - g.t_flag;
    g.t_st1 = (int)c->h_t1.size();
    if (g.dim == 1)
      for (int q : g.insts)
        for (int s = 0; s < c->probs[q].nx; s += kFused1)
          c->h_t1.push_back(mr_tile1{q, s, std::min(kFused1, c->probs[q].nx - s), 0});
    g.n_st1 = (int)c->h_t1.size() - g.t_st1;
    g.t_st2 = (int)c->h_t2.size();
    if (g.dim == 2) {
      /* largest instances first so the tail of the launch is short */
      std::vector<int> order = g.insts;
      std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        return plane_of(c->probs[a]) > plane_of(c->probs[b]); });
      for (int q : order) {
        const auto& p = c->probs[q];
        const size_t first = c->h_t2.size();
        const int w = strip_cells(p) - 2;
        const int rows = std::max(kMinRows, c->rows2);
        const bool lx = side_data(p, 0), rx = side_data(p, 1);
        if (!lx && !rx) {
          for (int y0 = 0; y0 < p.ny; y0 += rows)
            for (int x0 = 0; x0 < p.nx; x0 += w)
              c->h_t2.push_back(mr_tile2{q, x0, y0, std::min(rows, p.ny - y0)});
          xcd_order(c->h_t2, first, c->nxcd);
          continue;
        }
        /* strips whose staged columns (x0-3 .. x0+w+2) reach a left or right
           side with boundary data write those ghosts in every row step: half
           the rows, so that they finish with the rest of the launch */
        for (int x0 = 0; x0 < p.nx; x0 += w) {
          const bool edge = (lx && x0 - 3 < 0) || (rx && x0 + w + 2 >= p.nx);
          const int r = edge ? std::max(kMinRows, rows / 2) : rows;
          for (int y0 = 0; y0 < p.ny; y0 += r) c->h_t2.push_back(mr_tile2{q, x0, y0, std::min(r, p.ny - y0)});
        }
        xcd_order(c->h_t2, first, c->nxcd);
      }
    }
    g.n_st2 = (int)c->h_t2.size() - g.t_st2;
    g.t_kx = (int)c->h_t2.size();
    for (int q : g.insts) add_kx_tiles_if(c->h_t2, q, c->probs[q], false, c->kx_rows2, c->nxcd);
    g.n_kx = (int)c->h_t2.size() - g.t_kx;
    g.t_tvb = (int)c->h_t2.size();
    for (int q : g.insts) add_kx_tiles_if(c->h_t2, q, c->probs[q], true, c->kx_rows2, c->nxcd);
    g.n_tvb = (int)c->h_t2.size() - g.t_tvb;
  }
}

static mrhweno_status upload_lists(mrhweno_ctx* c) {
  MR_CHECK(c, hipMemcpy(c->t1, c->h_t1.data(), sizeof(mr_tile1) * std::max<size_t>(c->h_t1.size(), 1) , hipMemcpyHostToDevice));
  if (!c->h_t2.empty())
    MR_CHECK(c, hipMemcpy(c->t2, c->h_t2.data(), sizeof(mr_tile2) * c->h_t2.size(), hipMemcpyHostToDevice));
  return MRHWENO_OK;
}

static mrhweno_status pull(mrhweno_ctx* c);

/* Event hooks of the profiling mode: called between kernel classes. */
struct mr_prof {
  hipEvent_t ev[64];
  int cls[64];
  int n = 0;
};

static hipError_t mark(mrhweno_ctx* c, mr_prof* P, int cls) {
  if (!P) return hipSuccess;
  if (P->n >= 64) return hipErrorInvalidValue;
  P->cls[P->n] = cls;
  return hipEventRecord(P->ev[P->n++], c->stream);
}

/* the kernels of one SSP-RK3 step, in order; with P, an event is recorded
   after every kernel class (class ids: 0 reduce/dt, 1 summary, 2 flags,
   3 stage) */
static hipError_t enqueue_step(mrhweno_ctx* c, mr_prof* P = nullptr) {
  hipError_t e;
  hipStream_t s = c->stream;
  if ((e = mark(c, P, -1)) != hipSuccess) return e;
  if ((e = mr_launch_reduce(s, c->d, c->t1 + c->t_reduce, c->n_reduce, 0)) != hipSuccess) return e;
  if ((e = mr_launch_finalize(s, c->d, c->n, 0)) != hipSuccess) return e;
  if (c->any_learned && (e = mr_launch_fb_reset(s, c->cnt, 0)) != hipSuccess) return e;
  if ((e = mark(c, P, 0)) != hipSuccess) return e;
  for (int st = 0; st < 3; ++st) {
    if (st > 0 && c->any_lf) {
      if ((e = mr_launch_reduce(s, c->d, c->t1 + c->t_reduce, c->n_reduce, st)) != hipSuccess) return e;
      if ((e = mark(c, P, 0)) != hipSuccess) return e;
    }
    bool any = false;
    for (auto& g : c->groups)
      if (g.any_summ) {
        any = true;
        if ((e = mr_launch_summary(s, g.dim, g.bp, g.gb, c->d, c->t1 + g.t_summ, g.n_summ, st)) != hipSuccess) return e;
      }
    for (auto& g : c->groups) {
      if (g.n_kx > 0) {
        any = true;
        if ((e = mr_launch_kxrcf2(s, g.nc == 4 ? (g.ch ? 4 : 3) : 1, g.bp, g.gb, c->d, c->t2 + g.t_kx, g.n_kx, st)) !=
            hipSuccess)
          return e;
      }
      if (g.n_tvb > 0) {   /* the TVB test reads the indicator variable only */
        any = true;
        if ((e = mr_launch_kxrcf2(s, 1, g.bp, g.gb, c->d, c->t2 + g.t_tvb, g.n_tvb, st)) != hipSuccess) return e;
      }
    }
    if (c->any_learned) {
      any = true;
      if ((e = mr_launch_learned(s, c->d, c->tl, c->n_tl, st, c->lw, c->band, c->cnt, c->grid_l)) != hipSuccess)
        return e;
    }
    if (any && (e = mark(c, P, 1)) != hipSuccess) return e;
    for (auto& g : c->groups)
      if (g.n_flag > 0 && (e = mr_launch_flags(s, g.dim, c->d, c->t1 + g.t_flag, g.n_flag, st)) != hipSuccess) return e;
    if (c->any_learned &&
        (e = mr_launch_fallback(s, c->d, c->band, c->cnt, st, c->grid_fb, c->learned_bp)) != hipSuccess)
      return e;
    if ((e = mark(c, P, 2)) != hipSuccess) return e;
    for (auto& g : c->groups) {
      if (g.dim == 1) e = mr_launch_fused1(s, g.nc, g.bp, g.gb, c->d, c->t1 + g.t_st1, g.n_st1, st);
      else e = mr_launch_stage2(s, g.nc, g.bp, g.gb, g.ch, c->d, c->t2 + g.t_st2, g.n_st2, st, c->grid2);
      if (e != hipSuccess) return e;
    }
    if ((e = mark(c, P, 3)) != hipSuccess) return e;
  }
  return hipSuccess;
}

static mrhweno_status rebuild_graph(mrhweno_ctx* c) {
  if (c->exec) { (void)hipGraphExecDestroy(c->exec); c->exec = nullptr; }
  if (c->graph) { (void)hipGraphDestroy(c->graph); c->graph = nullptr; }
  if (!c->stream) return MRHWENO_OK;   /* the legacy default stream cannot be captured */
  if (c->any_learned && !c->weights_set) return MRHWENO_OK;   /* captured once weights are set */
  MR_CHECK(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
  hipError_t e = enqueue_step(c);
  hipGraph_t g = nullptr;
  hipError_t e2 = hipStreamEndCapture(c->stream, &g);
  if (e != hipSuccess) return fail(c, MRHWENO_ERR_DEVICE, std::string("capture: ") + hipGetErrorString(e));
  if (e2 != hipSuccess) return fail(c, MRHWENO_ERR_DEVICE, std::string("end capture: ") + hipGetErrorString(e2));
  c->graph = g;
  MR_CHECK(c, hipGraphInstantiate(&c->exec, c->graph, nullptr, nullptr, 0));
  return MRHWENO_OK;
}

extern "C" {

size_t mrhweno_workspace_bytes(const mrhweno_problem* probs, int n) {
  if (!probs || n <= 0) return 0;
  for (int q = 0; q < n; ++q)
    if (!validate(probs[q]).empty()) return 0;
  return layout(probs, n).total;
}

mrhweno_status mrhweno_create(const mrhweno_problem* probs, int n, void* const* moments_dev,
                              void* workspace_dev, void* hip_stream, mrhweno_ctx** out) {
  if (!out) return fail(nullptr, MRHWENO_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!probs || n <= 0 || !moments_dev || !workspace_dev)
    return fail(nullptr, MRHWENO_ERR_INVALID_ARG, "NULL argument or no instances");
  for (int q = 0; q < n; ++q) {
    std::string m = validate(probs[q]);
    if (!m.empty()) return fail(nullptr, MRHWENO_ERR_INVALID_ARG, "instance " + std::to_string(q) + ": " + m);
    if (!moments_dev[q]) return fail(nullptr, MRHWENO_ERR_INVALID_ARG, "NULL moments for instance " + std::to_string(q));
    if ((reinterpret_cast<uintptr_t>(moments_dev[q]) & 7) != 0)
      return fail(nullptr, MRHWENO_ERR_INVALID_ARG, "moments must be 8-byte aligned");
  }
  if ((reinterpret_cast<uintptr_t>(workspace_dev) & 255) != 0)
    return fail(nullptr, MRHWENO_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
  auto* c = new mrhweno_ctx();
  c->n = n;
  c->stream = (hipStream_t)hip_stream;
  c->ws = (char*)workspace_dev;
  c->probs.assign(probs, probs + n);
  c->L = layout(probs, n);
  c->d = (mr_inst*)(c->ws + c->L.insts);
  c->t1 = (mr_tile1*)(c->ws + c->L.tiles1);
  c->t2 = (mr_tile2*)(c->ws + c->L.tiles2);
  c->h.resize(n + 1);
  for (int q = 0; q < n; ++q) {
    const auto& p = probs[q];
    mr_inst& I = c->h[q];
    fill_inst(p, I);
    I.buf[0] = (double*)moments_dev[q];
    I.buf[1] = (double*)(c->ws + c->L.buf1[q]);
    I.buf[2] = (double*)(c->ws + c->L.buf2[q]);
    I.unm = p.dim == 2 ? (double*)(c->ws + c->L.unm[q]) : nullptr;
    I.flags[0] = (unsigned char*)(c->ws + c->L.fl0[q]);
    I.flags[1] = (unsigned char*)(c->ws + c->L.fl1[q]);
    I.summ = needs_summ(p) ? (double*)(c->ws + c->L.summ[q]) : nullptr;
    I.aleph = nullptr;
    I.cur = 0;
    if (p.flux == MRHWENO_BURGERS_LF) c->any_lf = true;
  }
  std::memset(&c->h[n], 0, sizeof(mr_inst));
  {
    int dev = 0, nx = 1;
    if (hipGetDevice(&dev) == hipSuccess && hipDeviceGetAttribute(&nx, hipDeviceAttributeNumberOfXccs, dev) == hipSuccess &&
        nx >= 1 && nx <= 64)
      c->nxcd = nx;
  }
  /* learned indicator: work items, band list, counters */
  if (c->L.n_tilesl) {
    c->any_learned = true;
    c->lw = (mr_learn_w*)(c->ws + c->L.lw);
    c->cnt = (int*)(c->ws + c->L.cnt);
    c->band = (mr_band*)(c->ws + c->L.band);
    c->tl = (mr_tile2*)(c->ws + c->L.tilesl);
    std::vector<mr_tile2> tl;
    for (int q = 0; q < n; ++q)
      if (learned(probs[q])) {
        add_learn_tiles(tl, q, probs[q]);
        c->learned_bp |= probs[q].beta_on;
      }
    c->n_tl = (int)tl.size();
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0) {
      c->grid_l = 2 * cus;    /* two work groups of the fused kernel per CU */
      c->grid_fb = 4 * cus;
    }
    if (hipMemcpy(c->tl, tl.data(), sizeof(mr_tile2) * tl.size(), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemset(c->cnt, 0, 16 * sizeof(int)) != hipSuccess) {
      delete c;
      return fail(nullptr, MRHWENO_ERR_DEVICE, "learned-indicator set-up failed");
    }
  }
  /* launch groups */
  for (int q = 0; q < n; ++q) {
    const auto& p = probs[q];
    const int nc = ncomp_of(p);
    Group* gp = nullptr;
    const int ch = p.dim == 2 && p.charwise;
    for (auto& g : c->groups)
      if (g.dim == p.dim && g.nc == nc && g.bp == p.beta_on && g.gb == gb_of(c->h[q]) && g.ch == ch) gp = &g;
    if (!gp) { c->groups.push_back(Group{p.dim, nc, p.beta_on, gb_of(c->h[q]), ch}); gp = &c->groups.back(); }
    gp->insts.push_back(q);
    gp->any_summ |= needs_summ(p);
  }
  build_lists(c);
  mrhweno_status st;
  /* flag planes start cleared (read before the first step by the probes and
     the autotuner) */
  for (int q = 0; q < n; ++q) {
    for (int f = 0; f < 2; ++f)
      if (hipMemset(c->h[q].flags[f], 0, (size_t)c->h[q].fex * c->h[q].fey) != hipSuccess) {
        delete c;
        return fail(nullptr, MRHWENO_ERR_DEVICE, "flag plane clear failed");
      }
  }
  if (hipMemcpy(c->d, c->h.data(), sizeof(mr_inst) * (n + 1), hipMemcpyHostToDevice) != hipSuccess) {
    delete c;
    return fail(nullptr, MRHWENO_ERR_DEVICE, "descriptor upload failed");
  }
  if ((st = upload_lists(c)) != MRHWENO_OK || (st = rebuild_graph(c)) != MRHWENO_OK) {
    std::string m = c->err;
    mrhweno_destroy(c);
    return fail(nullptr, st, m);
  }
  *out = c;
  return MRHWENO_OK;
}

mrhweno_status mrhweno_set_launch(mrhweno_ctx* c, int rows_2d, int grid_2d) {
  if (!c) return fail(nullptr, MRHWENO_ERR_INVALID_ARG, "NULL context");
  if (rows_2d < kMinRows || rows_2d > 4096 || grid_2d < 0)
    return fail(c, MRHWENO_ERR_INVALID_ARG, "rows_2d must be in [8, 4096], grid_2d >= 0");
  MR_CHECK(c, hipStreamSynchronize(c->stream));
  c->rows2 = rows_2d;
  c->grid2 = grid_2d;
  build_lists(c);
  mrhweno_status st = upload_lists(c);
  if (st != MRHWENO_OK) return st;
  return rebuild_graph(c);
}

mrhweno_status mrhweno_step(mrhweno_ctx* c, int nsteps) {
  if (!c) return fail(nullptr, MRHWENO_ERR_INVALID_ARG, "NULL context");
  if (nsteps < 0) return fail(c, MRHWENO_ERR_INVALID_ARG, "nsteps < 0");
  if (c->any_learned && !c->weights_set)
    return fail(c, MRHWENO_ERR_NOT_READY, "learned indicator has no weights (mrhweno_set_indicator)");
  for (int k = 0; k < nsteps; ++k) {
    if (c->exec) MR_CHECK(c, hipGraphLaunch(c->exec, c->stream));
    else MR_CHECK(c, enqueue_step(c));
  }
  return MRHWENO_OK;
}

mrhweno_status mrhweno_autotune(mrhweno_ctx* c, const int* rows_cand, int n_rows, const int* grid_cand, int n_grid,
                                int reps, int* best_rows, int* best_grid, float* best_ms) {
  if (!c || !rows_cand || n_rows <= 0 || reps <= 0 || (n_grid > 0 && !grid_cand))
    return fail(c, MRHWENO_ERR_INVALID_ARG, "bad autotune arguments");
  for (int a = 0; a < n_rows; ++a)
    if (rows_cand[a] < kMinRows || rows_cand[a] > 4096) return fail(c, MRHWENO_ERR_INVALID_ARG, "rows candidate out of range");
  mrhweno_status st = pull(c);
  if (st != MRHWENO_OK) return st;
  bool any2d = false;
  for (auto& g : c->groups) any2d |= g.dim == 2;
  if (!any2d) {
    if (best_rows) *best_rows = c->rows2;
    if (best_grid) *best_grid = c->grid2;
    if (best_ms) *best_ms = 0.0f;
    return MRHWENO_OK;
  }
  /* residual-only descriptors: input = current state, output = a free
     rotation buffer; the real descriptors are restored afterwards */
  std::vector<mr_inst> saved = c->h;
  std::vector<mr_inst> tmp = c->h;
  for (int q = 0; q < c->n; ++q) {
    mr_inst& I = tmp[q];
    const int cur = I.cur;
    I.p_in[0] = I.buf[cur];
    I.p_un = I.buf[cur];
    I.p_out[0] = I.buf[(cur + 1) % 3];
    I.lfa[0] = I.lfa[0] ? I.lfa[0] : 0x3ff0000000000000ull;   /* any alpha: only the time matters */
  }
  MR_CHECK(c, hipMemcpy(c->d, tmp.data(), sizeof(mr_inst) * c->n, hipMemcpyHostToDevice));
  hipEvent_t e0, e1;
  MR_CHECK(c, hipEventCreate(&e0));
  MR_CHECK(c, hipEventCreate(&e1));
  const int saved_rows = c->rows2, saved_grid = c->grid2;
  float best = 1e30f;
  int br = saved_rows, bg = saved_grid;
  const int ng = n_grid > 0 ? n_grid : 1;
  for (int a = 0; a < n_rows && st == MRHWENO_OK; ++a)
    for (int b = 0; b < ng && st == MRHWENO_OK; ++b) {
      c->rows2 = rows_cand[a];
      c->grid2 = n_grid > 0 ? grid_cand[b] : 0;
      build_lists(c);
      if ((st = upload_lists(c)) != MRHWENO_OK) break;
      auto launch = [&]() -> hipError_t {
        for (auto& g : c->groups)
          if (g.dim == 2) {
            hipError_t e = mr_launch_stage2(c->stream, g.nc, g.bp, g.gb, g.ch, c->d, c->t2 + g.t_st2, g.n_st2, 3,
                                            c->grid2);
            if (e != hipSuccess) return e;
          }
        return hipSuccess;
      };
      if (launch() != hipSuccess) { st = fail(c, MRHWENO_ERR_DEVICE, "autotune launch"); break; }
      (void)hipEventRecord(e0, c->stream);
      for (int r = 0; r < reps; ++r)
        if (launch() != hipSuccess) { st = fail(c, MRHWENO_ERR_DEVICE, "autotune launch"); break; }
      (void)hipEventRecord(e1, c->stream);
      if (hipEventSynchronize(e1) != hipSuccess) { st = fail(c, MRHWENO_ERR_DEVICE, "autotune sync"); break; }
      float ms = 0.0f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      ms /= reps;
      if (ms < best) { best = ms; br = c->rows2; bg = c->grid2; }
    }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  /* restore the descriptors and apply the choice */
  c->h = saved;
  if (hipMemcpy(c->d, c->h.data(), sizeof(mr_inst) * c->n, hipMemcpyHostToDevice) != hipSuccess && st == MRHWENO_OK)
    st = fail(c, MRHWENO_ERR_DEVICE, "descriptor restore");
  c->rows2 = st == MRHWENO_OK ? br : saved_rows;
  c->grid2 = st == MRHWENO_OK ? bg : saved_grid;
  build_lists(c);
  mrhweno_status s2 = upload_lists(c);
  if (st == MRHWENO_OK) st = s2;
  if (st == MRHWENO_OK) st = rebuild_graph(c);
  if (best_rows) *best_rows = c->rows2;
  if (best_grid) *best_grid = c->grid2;
  if (best_ms) *best_ms = best;
  return st;
}

mrhweno_status mrhweno_set_indicator_launch(mrhweno_ctx* c, int rows) {
  if (!c) return fail(nullptr, MRHWENO_ERR_INVALID_ARG, "NULL context");
  if (rows != 0 && (rows < kKxMinRows || rows > kKxMaxRows))
    return fail(c, MRHWENO_ERR_INVALID_ARG, "indicator rows must be 0 or in [8, 256]");
  MR_CHECK(c, hipStreamSynchronize(c->stream));
  c->kx_rows2 = rows;
  build_lists(c);
  mrhweno_status st = upload_lists(c);
  if (st != MRHWENO_OK) return st;
  return rebuild_graph(c);
}

mrhweno_status mrhweno_autotune_indicator(mrhweno_ctx* c, const int* rows_cand, int n_rows, int reps,
                                          int* best_rows, float* best_ms) {
  if (!c || !rows_cand || n_rows <= 0 || reps <= 0) return fail(c, MRHWENO_ERR_INVALID_ARG, "bad autotune arguments");
  for (int a = 0; a < n_rows; ++a)
    if (rows_cand[a] != 0 && (rows_cand[a] < kKxMinRows || rows_cand[a] > kKxMaxRows))
      return fail(c, MRHWENO_ERR_INVALID_ARG, "indicator rows candidate neither 0 nor in [8, 256]");
  MR_CHECK(c, hipStreamSynchronize(c->stream));
  mrhweno_status st = MRHWENO_OK;
  if (st != MRHWENO_OK) return st;
  bool any = false;
  for (auto& g : c->groups) any |= g.n_kx > 0;
  if (!any) {
    if (best_rows) *best_rows = c->kx_rows2;
    if (best_ms) *best_ms = 0.0f;
    return MRHWENO_OK;
  }
  hipEvent_t e0, e1;
  MR_CHECK(c, hipEventCreate(&e0));
  MR_CHECK(c, hipEventCreate(&e1));
  const int saved = c->kx_rows2;
  float best = 1e30f;
  int br = saved;
  for (int a = 0; a < n_rows && st == MRHWENO_OK; ++a) {
    c->kx_rows2 = rows_cand[a];
    build_lists(c);
    if ((st = upload_lists(c)) != MRHWENO_OK) break;
    /* one-off evaluations (stage 3) of the KXRCF pass on rotation buffer 0,
       which always holds a state of the instance; they write the first
       flag plane only, which every step rewrites before reading it */
    auto launch = [&]() -> hipError_t {
      for (auto& g : c->groups)
        if (g.n_kx > 0) {
          hipError_t e = mr_launch_kxrcf2(c->stream, g.nc == 4 ? (g.ch ? 4 : 3) : 1, g.bp, g.gb, c->d, c->t2 + g.t_kx,
                                          g.n_kx, 3);
          if (e != hipSuccess) return e;
        }
      return hipSuccess;
    };
    if (launch() != hipSuccess) { st = fail(c, MRHWENO_ERR_DEVICE, "autotune launch"); break; }
    (void)hipEventRecord(e0, c->stream);
    for (int r = 0; r < reps; ++r)
      if (launch() != hipSuccess) { st = fail(c, MRHWENO_ERR_DEVICE, "autotune launch"); break; }
    (void)hipEventRecord(e1, c->stream);
    if (hipEventSynchronize(e1) != hipSuccess) { st = fail(c, MRHWENO_ERR_DEVICE, "autotune sync"); break; }
    float ms = 0.0f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    ms /= reps;
    if (ms < best) { best = ms; br = c->kx_rows2; }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  c->kx_rows2 = st == MRHWENO_OK ? br : saved;
  build_lists(c);
  mrhweno_status s2 = upload_lists(c);
  if (st == MRHWENO_OK) st = s2;
  if (st == MRHWENO_OK) st = rebuild_graph(c);
  if (best_rows) *best_rows = c->kx_rows2;
  if (best_ms) *best_ms = best;
  return st;
}

mrhweno_status mrhweno_profile(mrhweno_ctx* c, int nsteps, float* ms_out, int* launches_out) {
  if (!c || !ms_out || nsteps < 0) return fail(c, MRHWENO_ERR_INVALID_ARG, "bad argument");
  if (c->any_learned && !c->weights_set)
    return fail(c, MRHWENO_ERR_NOT_READY, "learned indicator has no weights (mrhweno_set_indicator)");
  for (int k = 0; k < 4; ++k) { ms_out[k] = 0.0f; if (launches_out) launches_out[k] = 0; }
  mr_prof P;
  for (int k = 0; k < 64; ++k) MR_CHECK(c, hipEventCreate(&P.ev[k]));
  mrhweno_status st = MRHWENO_OK;
  for (int it = 0; it < nsteps && st == MRHWENO_OK; ++it) {
    P.n = 0;
    hipError_t e = enqueue_step(c, &P);
    if (e != hipSuccess) { st = fail(c, MRHWENO_ERR_DEVICE, std::string("profile: ") + hipGetErrorString(e)); break; }
    if (hipEventSynchronize(P.ev[P.n - 1]) != hipSuccess) { st = fail(c, MRHWENO_ERR_DEVICE, "event sync"); break; }
    for (int k = 1; k < P.n; ++k) {
      float ms = 0.0f;
      if (hipEventElapsedTime(&ms, P.ev[k - 1], P.ev[k]) != hipSuccess) { st = fail(c, MRHWENO_ERR_DEVICE, "event time"); break; }
      ms_out[P.cls[k]] += ms;
      if (launches_out) launches_out[P.cls[k]] += 1;
    }
  }
  for (int k = 0; k < 64; ++k) (void)hipEventDestroy(P.ev[k]);
  return st;
}

static mrhweno_status pull(mrhweno_ctx* c) {
  MR_CHECK(c, hipStreamSynchronize(c->stream));
  MR_CHECK(c, hipMemcpy(c->h.data(), c->d, sizeof(mr_inst) * c->n, hipMemcpyDeviceToHost));
  return MRHWENO_OK;
}

mrhweno_status mrhweno_sync(mrhweno_ctx* c, double* t_out, long* steps_out) {
  if (!c) return fail(nullptr, MRHWENO_ERR_INVALID_ARG, "NULL context");
  mrhweno_status st = pull(c);
  if (st != MRHWENO_OK) return st;
  bool bad = false;
  for (int q = 0; q < c->n; ++q) {
    mr_inst& I = c->h[q];
    if (I.cur != 0) {
      MR_CHECK(c, hipMemcpyAsync(I.buf[0], I.buf[I.cur], state_bytes(c->probs[q]), hipMemcpyDeviceToDevice, c->stream));
      I.cur = 0;
      MR_CHECK(c, hipMemcpyAsync(&c->d[q].cur, &I.cur, sizeof(int), hipMemcpyHostToDevice, c->stream));
      MR_CHECK(c, hipStreamSynchronize(c->stream));
    }
    if (t_out) t_out[q] = I.t;
    if (steps_out) steps_out[q] = (long)I.steps;
    bad |= I.err != 0;
  }
  if (bad) return fail(c, MRHWENO_ERR_NONPHYSICAL, "non-physical or non-finite state met; rolled back to the last good step");
  return MRHWENO_OK;
}

mrhweno_status mrhweno_set_time(mrhweno_ctx* c, int q, double t, long steps) {
  if (!c) return fail(nullptr, MRHWENO_ERR_INVALID_ARG, "NULL context");
  if (q < 0 || q >= c->n || !(t >= 0.0) || steps < 0) return fail(c, MRHWENO_ERR_INVALID_ARG, "bad instance, time or step count");
  mrhweno_status st = pull(c);
  if (st != MRHWENO_OK) return st;
  c->h[q].t = t;
  c->h[q].steps = steps;
  c->h[q].err = 0;
  c->h[q].rolled = 0;
  MR_CHECK(c, hipMemcpy(&c->d[q], &c->h[q], sizeof(mr_inst), hipMemcpyHostToDevice));
  return MRHWENO_OK;
}

mrhweno_status mrhweno_last_dt(mrhweno_ctx* c, double* dt_out) {
  if (!c || !dt_out) return fail(c, MRHWENO_ERR_INVALID_ARG, "NULL argument");
  mrhweno_status st = pull(c);
  if (st != MRHWENO_OK) return st;
  for (int q = 0; q < c->n; ++q) dt_out[q] = c->h[q].dt;
  return MRHWENO_OK;
}

/* Work lists of a one-off evaluation of the instance in descriptor slot
   `slot`: per-cell chunks (reduction, 1D face summaries, flags, values,
   1D stage), 2D stage strips, and the learned or fused 2D KXRCF/TVB
   strips. */
struct ProbeLists {
  std::vector<mr_tile1> t1;
  std::vector<mr_tile2> t2, t3;
  int n_red = 0, t_sum = 0, n_sum = 0, t_flg = 0, n_flg = 0, t_val = 0, n_val = 0, t_st = 0, n_st = 0;
  bool kx2 = false;
};

static ProbeLists probe_lists(const mrhweno_problem& p, int slot) {
  ProbeLists L;
  const bool lrn = learned(p);
  add_cells(L.t1, slot, plane_of(p));
  L.n_red = (int)L.t1.size();
  L.t_sum = (int)L.t1.size();
  if (needs_summ(p)) add_cells(L.t1, slot, (long long)sex(p) * sey(p));
  L.n_sum = (int)L.t1.size() - L.t_sum;
  L.t_flg = (int)L.t1.size();
  L.kx2 = kx_tiles(p) > 0;   /* 2D KXRCF / TVB: flags from the fused kernel */
  if (!lrn && !L.kx2) add_cells(L.t1, slot, (long long)fex(p) * fey(p));
  L.n_flg = (int)L.t1.size() - L.t_flg;
  L.t_val = (int)L.t1.size();
  add_cells(L.t1, slot, plane_of(p));
  L.n_val = (int)L.t1.size() - L.t_val;
  L.t_st = (int)L.t1.size();
  if (p.dim == 1) {
    for (int s = 0; s < p.nx; s += kBlock - 2) L.t1.push_back(mr_tile1{slot, s, std::min(kBlock - 2, p.nx - s), 0});
  } else {
    const int w = strip_cells(p) - 2;
    for (int y0 = 0; y0 < p.ny; y0 += 32)
      for (int x0 = 0; x0 < p.nx; x0 += w) L.t2.push_back(mr_tile2{slot, x0, y0, std::min(32, p.ny - y0)});
  }
  L.n_st = (int)L.t1.size() - L.t_st;
  if (lrn) add_learn_tiles(L.t3, slot, p);
  if (L.kx2) add_kx_tiles(L.t3, slot, p);
  return L;
}

/* bytes of the device copies of a probe's lists (three 256-byte aligned
   pieces) */
static size_t probe_list_bytes(const ProbeLists& L, size_t* o2, size_t* o3) {
  *o2 = al(sizeof(mr_tile1) * L.t1.size());
  *o3 = *o2 + al(sizeof(mr_tile2) * std::max<size_t>(L.t2.size(), 1));
  return *o3 + sizeof(mr_tile2) * std::max<size_t>(L.t3.size(), 1);
}

/* The kernels of a one-off evaluation of a non-learned instance whose
   descriptor sits in d[slot] and whose lists were copied to d1/d2/d3:
   wave speeds and dt, troubled cells (Step 2.1), then the final values
   (kind 0, into out) or L(U) (kind 2, into the descriptor's p_out[0]). */
static hipError_t probe_kernels(hipStream_t s, const mrhweno_problem& p, const mr_inst& I, mr_inst* d, int slot,
                                const ProbeLists& L, const mr_tile1* d1, const mr_tile2* d2, const mr_tile2* d3,
                                int kind, void* out) {
  hipError_t e;
  mr_tile1* t1 = const_cast<mr_tile1*>(d1);
  mr_tile2* t2 = const_cast<mr_tile2*>(d2);
  mr_tile2* t3 = const_cast<mr_tile2*>(d3);
  if ((e = mr_launch_reduce(s, d, t1, L.n_red, 0)) != hipSuccess) return e;
  if ((e = mr_launch_finalize(s, d + slot, 1, 1)) != hipSuccess) return e;
  if ((e = mr_launch_summary(s, p.dim, p.beta_on, gb_of(I), d, t1 + L.t_sum, L.n_sum, 3)) != hipSuccess) return e;
  if ((e = mr_launch_flags(s, p.dim, d, t1 + L.t_flg, L.n_flg, 3)) != hipSuccess) return e;
  const int ch = p.dim == 2 && p.charwise;
  if (L.kx2 && (e = mr_launch_kxrcf2(s, ncomp_of(p) == 4 && !tvb(p) ? (ch ? 4 : 3) : 1, p.beta_on, gb_of(I), d,
                                     t3, (int)L.t3.size(), 3)) != hipSuccess)
    return e;
  const int nc = ncomp_of(p);
  if (kind == 0 && (e = mr_launch_values(s, p.dim, nc, p.beta_on, d, t1 + L.t_val, L.n_val, (double*)out)) != hipSuccess)
    return e;
  if (kind == 2) {
    if (p.dim == 1) e = mr_launch_stage1(s, nc, p.beta_on, gb_of(I), d, t1 + L.t_st, L.n_st, 3, 0);
    else e = mr_launch_stage2(s, nc, p.beta_on, gb_of(I), ch, d, t2, (int)L.t2.size(), 3, 0);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

/* kind: 0 = reconstruct, 1 = flag, 2 = residual, 3 = learned-indicator
   decisions (out = decision plane, may be NULL) */
static mrhweno_status probe(mrhweno_ctx* c, int q, const void* U, void* out, void* flags, void* aleph, int kind) {
  if (!c) return fail(nullptr, MRHWENO_ERR_INVALID_ARG, "NULL context");
  if (q < 0 || q >= c->n || !U) return fail(c, MRHWENO_ERR_INVALID_ARG, "bad instance or NULL state");
  if ((kind == 0 || kind == 2) && !out) return fail(c, MRHWENO_ERR_INVALID_ARG, "NULL output");
  const auto& p = c->probs[q];
  const bool lrn = learned(p);
  if (lrn && !c->weights_set)
    return fail(c, MRHWENO_ERR_NOT_READY, "learned indicator has no weights (mrhweno_set_indicator)");
  if (kind == 3 && !lrn) return fail(c, MRHWENO_ERR_INVALID_ARG, "instance does not use the learned indicator");
  if (aleph && !kxrcf(p))
    return fail(c, MRHWENO_ERR_UNSUPPORTED, "KXRCF ratios are formed for KXRCF instances only");
  mrhweno_status st = pull(c);   /* the probe reuses the instance's scratch planes */
  if (st != MRHWENO_OK) return st;
  mr_inst I = c->h[q];
  I.buf[0] = (double*)U;
  I.cur = 0;
  I.p_in[0] = (const double*)U;
  I.p_un = (const double*)U;
  I.p_out[0] = (double*)out;
  I.active = 1; I.err = 0; I.rolled = 0;
  I.amax[0] = I.amax[1] = 0ull;
  I.lfa[0] = I.lfa[1] = I.lfa[2] = 0ull;
  I.dt = 0.0;
  double* al_buf = (double*)(c->ws + c->L.probe_aleph);
  I.aleph = aleph ? al_buf : nullptr;
  const int slot = c->n;
  const ProbeLists PL = probe_lists(p, slot);
  /* the probe area holds the 1D list, the 2D list and the learned or the
     2D KXRCF list */
  char* area = c->ws + c->L.probe_tiles;
  size_t o2 = 0, o3 = 0;
  if (probe_list_bytes(PL, &o2, &o3) > sizeof(mr_tile2) * (c->L.n_probe_tiles + 64))
    return fail(c, MRHWENO_ERR_DEVICE, "probe list overflow");
  mr_tile1* d1 = (mr_tile1*)area;
  mr_tile2* d2 = (mr_tile2*)(area + o2);
  mr_tile2* d3 = (mr_tile2*)(area + o3);
  MR_CHECK(c, hipMemcpy(&c->d[slot], &I, sizeof(mr_inst), hipMemcpyHostToDevice));
  MR_CHECK(c, hipMemcpy(d1, PL.t1.data(), sizeof(mr_tile1) * PL.t1.size(), hipMemcpyHostToDevice));
  if (!PL.t2.empty()) MR_CHECK(c, hipMemcpy(d2, PL.t2.data(), sizeof(mr_tile2) * PL.t2.size(), hipMemcpyHostToDevice));
  if (!PL.t3.empty()) MR_CHECK(c, hipMemcpy(d3, PL.t3.data(), sizeof(mr_tile2) * PL.t3.size(), hipMemcpyHostToDevice));
  hipStream_t s = c->stream;
  const size_t frow = (size_t)(p.dim == 2 ? kFHalo : 0) * I.fex + kFHalo;   /* first interior flag */
  if (lrn) {
    MR_CHECK(c, mr_launch_reduce(s, c->d, d1, PL.n_red, 0));
    MR_CHECK(c, mr_launch_finalize(s, c->d + slot, 1, 1));
    MR_CHECK(c, mr_launch_fb_reset(s, c->cnt, 1));
    MR_CHECK(c, mr_launch_learned(s, c->d, d3, (int)PL.t3.size(), 3, c->lw, c->band, c->cnt, c->grid_l));
    if (kind == 3 && out)
      MR_CHECK(c, hipMemcpy2DAsync(out, p.nx, I.flags[0] + frow, I.fex, p.nx, p.ny, hipMemcpyDeviceToDevice, s));
    MR_CHECK(c, mr_launch_fallback(s, c->d, c->band, c->cnt, 3, c->grid_fb, p.beta_on));
    const int nc = ncomp_of(p);
    if (kind == 0) MR_CHECK(c, mr_launch_values(s, p.dim, nc, p.beta_on, c->d, d1 + PL.t_val, PL.n_val, (double*)out));
    if (kind == 2) MR_CHECK(c, mr_launch_stage2(s, nc, p.beta_on, gb_of(I), 0, c->d, d2, (int)PL.t2.size(), 3, 0));
  } else {
    MR_CHECK(c, probe_kernels(s, p, I, c->d, slot, PL, d1, d2, d3, kind, out));
  }
  if (flags)
    MR_CHECK(c, hipMemcpy2DAsync(flags, p.nx, I.flags[0] + frow, I.fex, p.nx, p.dim == 2 ? p.ny : 1,
                                 hipMemcpyDeviceToDevice, s));
  if (aleph)
    MR_CHECK(c, hipMemcpyAsync(aleph, al_buf, sizeof(double) * 2 * plane_of(p), hipMemcpyDeviceToDevice, s));
  MR_CHECK(c, hipStreamSynchronize(s));
  return MRHWENO_OK;
}

mrhweno_status mrhweno_reconstruct(mrhweno_ctx* c, int q, const void* U, void* gl, void* flags) {
  return probe(c, q, U, gl, flags, nullptr, 0);
}
mrhweno_status mrhweno_flag(mrhweno_ctx* c, int q, const void* U, void* flags, void* aleph) {
  if (!flags) return fail(c, MRHWENO_ERR_INVALID_ARG, "NULL flags");
  return probe(c, q, U, nullptr, flags, aleph, 1);
}
mrhweno_status mrhweno_residual(mrhweno_ctx* c, int q, const void* U, void* R, void* flags) {
  return probe(c, q, U, R, flags, nullptr, 2);
}

/* ---- L(U) without allocation: scratch in a file-scope device array ---- */
/* Per device, the descriptor, the work lists, the troubled-cell plane and
   the 1D face summaries of mrhweno_residual_noalloc live here.  Host code
   never passes this name to a kernel or a copy: it takes the array's
   device address from hipGetSymbolAddress once per device (each device
   holds its own copy) and uses that. */
static __device__ __align__(256) unsigned char scratch[MRHWENO_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned char* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

/* device address of `scratch` on the current device (set up on first use) */
static hipError_t scratch_ptr(unsigned char** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!ptr) return hipErrorInvalidSymbol;
    g_scratch_ptr[dev] = (unsigned char*)ptr;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

mrhweno_status mrhweno_residual_noalloc(const mrhweno_problem* pp, const void* U, void* R, void* flags,
                                        void* hip_stream) {
  if (!pp || !U || !R) return fail(nullptr, MRHWENO_ERR_INVALID_ARG, "NULL problem, state or residual");
  const mrhweno_problem& p = *pp;
  const std::string m = validate(p);
  if (!m.empty()) return fail(nullptr, MRHWENO_ERR_INVALID_ARG, m);
  if (learned(p)) return fail(nullptr, MRHWENO_ERR_UNSUPPORTED, "the learned indicator needs a context (mrhweno_create)");
  if ((reinterpret_cast<uintptr_t>(U) & 7) != 0 || (reinterpret_cast<uintptr_t>(R) & 7) != 0)
    return fail(nullptr, MRHWENO_ERR_INVALID_ARG, "state and residual must be 8-byte aligned");
  /* scratch layout: descriptor | lists | flag plane | 1D face summaries */
  const ProbeLists PL = probe_lists(p, 0);
  size_t o2 = 0, o3 = 0;
  const size_t o_lists = al(sizeof(mr_inst));
  const size_t o_fl = o_lists + al(probe_list_bytes(PL, &o2, &o3));
  const size_t o_summ = o_fl + al((size_t)fex(p) * fey(p));
  const size_t need = o_summ + (needs_summ(p) ? sizeof(double) * nsumm(p) * (size_t)sex(p) * sey(p) : 0);
  if (need > (size_t)MRHWENO_NOALLOC_SCRATCH_BYTES)
    return fail(nullptr, MRHWENO_ERR_INVALID_ARG,
                "problem needs " + std::to_string(need) + " bytes of scratch; the static scratch holds " +
                    std::to_string((size_t)MRHWENO_NOALLOC_SCRATCH_BYTES));
  unsigned char* base = nullptr;
  hipError_t e = scratch_ptr(&base);
  if (e != hipSuccess) return fail(nullptr, MRHWENO_ERR_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
  mr_inst I;
  fill_inst(p, I);
  I.buf[0] = (double*)U;
  I.p_in[0] = (const double*)U;
  I.p_un = (const double*)U;
  I.p_out[0] = (double*)R;
  I.flags[0] = I.flags[1] = base + o_fl;
  I.summ = needs_summ(p) ? (double*)(base + o_summ) : nullptr;
  I.active = 1;
  mr_inst* d = (mr_inst*)base;
  mr_tile1* d1 = (mr_tile1*)(base + o_lists);
  mr_tile2* d2 = (mr_tile2*)(base + o_lists + o2);
  mr_tile2* d3 = (mr_tile2*)(base + o_lists + o3);
  hipStream_t s = (hipStream_t)hip_stream;
#define MR_NA(expr)                                                                                    \
  do {                                                                                                 \
    hipError_t e_ = (expr);                                                                            \
    if (e_ != hipSuccess) return fail(nullptr, MRHWENO_ERR_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)
  /* every word the kernels read is written here or by an earlier kernel of
     this call: the descriptor and lists are copied in, the flag plane is
     written whole by the troubled-cell pass, the summaries by theirs */
  MR_NA(hipMemcpyAsync(d, &I, sizeof(mr_inst), hipMemcpyHostToDevice, s));
  MR_NA(hipMemcpyAsync(d1, PL.t1.data(), sizeof(mr_tile1) * PL.t1.size(), hipMemcpyHostToDevice, s));
  if (!PL.t2.empty()) MR_NA(hipMemcpyAsync(d2, PL.t2.data(), sizeof(mr_tile2) * PL.t2.size(), hipMemcpyHostToDevice, s));
  if (!PL.t3.empty()) MR_NA(hipMemcpyAsync(d3, PL.t3.data(), sizeof(mr_tile2) * PL.t3.size(), hipMemcpyHostToDevice, s));
  MR_NA(probe_kernels(s, p, I, d, 0, PL, d1, d2, d3, 2, R));
  if (flags) {
    const size_t frow = (size_t)(p.dim == 2 ? kFHalo : 0) * I.fex + kFHalo;
    MR_NA(hipMemcpy2DAsync(flags, p.nx, I.flags[0] + frow, I.fex, p.nx, p.dim == 2 ? p.ny : 1,
                           hipMemcpyDeviceToDevice, s));
  }
  /* the host lists above must outlive their copies */
  MR_NA(hipStreamSynchronize(s));
#undef MR_NA
  return MRHWENO_OK;
}

mrhweno_status mrhweno_indicator(mrhweno_ctx* c, int q, const void* U, void* decision, void* flags) {
  return probe(c, q, U, decision, flags, nullptr, 3);
}

mrhweno_status mrhweno_set_indicator(mrhweno_ctx* c, const void* params, double band_lo, double band_hi) {
  if (!c) return fail(nullptr, MRHWENO_ERR_INVALID_ARG, "NULL context");
  if (!params) return fail(c, MRHWENO_ERR_INVALID_ARG, "NULL parameters");
  if (!(band_lo >= 0.0) || !(band_hi <= 1.0) || !(band_lo <= band_hi))
    return fail(c, MRHWENO_ERR_INVALID_ARG, "band must satisfy 0 <= band_lo <= band_hi <= 1");
  if (!c->any_learned) return fail(c, MRHWENO_ERR_INVALID_ARG, "no instance uses the learned indicator");
  mrhweno_status st = pull(c);
  if (st != MRHWENO_OK) return st;
  MR_CHECK(c, mr_launch_pack(c->stream, params, c->lw));
  for (int q = 0; q < c->n; ++q) {
    c->h[q].band_lo = band_lo;
    c->h[q].band_hi = band_hi;
  }
  MR_CHECK(c, hipStreamSynchronize(c->stream));
  MR_CHECK(c, hipMemcpy(c->d, c->h.data(), sizeof(mr_inst) * c->n, hipMemcpyHostToDevice));
  c->weights_set = true;
  return rebuild_graph(c);
}

mrhweno_status mrhweno_features(mrhweno_ctx* c, int q, const void* U, const int* cells, int n, void* out) {
  if (!c) return fail(nullptr, MRHWENO_ERR_INVALID_ARG, "NULL context");
  if (q < 0 || q >= c->n || !U || !cells || !out || n < 0)
    return fail(c, MRHWENO_ERR_INVALID_ARG, "bad instance, count or NULL pointer");
  const auto& p = c->probs[q];
  if (p.dim != 2 || p.flux != MRHWENO_EULER_HLLC) return fail(c, MRHWENO_ERR_INVALID_ARG, "features are for 2D Euler");
  if (n == 0) return MRHWENO_OK;
  mrhweno_status st = pull(c);
  if (st != MRHWENO_OK) return st;
  mr_inst I = c->h[q];
  I.p_in[0] = (const double*)U;
  const int slot = c->n;
  MR_CHECK(c, hipMemcpy(&c->d[slot], &I, sizeof(mr_inst), hipMemcpyHostToDevice));
  MR_CHECK(c, mr_launch_features(c->stream, c->d, slot, cells, n, out));
  MR_CHECK(c, hipStreamSynchronize(c->stream));
  return MRHWENO_OK;
}

/* ---- network training (stateless; on the caller's stream) ---- */
int mrhweno_mlp_param_count(void) { return MR_NPARAM; }
int mrhweno_mlp_feature_count(void) { return MR_KP; }
size_t mrhweno_mlp_cache_bytes(int batch) { return mr_mlp_cache_bytes(batch); }

#define MR_MLP_CHECK(expr)                                                                     do {                                                                                           hipError_t e_ = (expr);                                                                      if (e_ != hipSuccess) return fail(nullptr, MRHWENO_ERR_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));   } while (0)

mrhweno_status mrhweno_mlp_gemm(void* stream, int M, int N, int K, const void* A, long long sAm, long long sAk,
                                const void* B, long long sBk, long long sBn, void* Cm, long long sCm, long long sCn) {
  if (M <= 0 || N <= 0 || K <= 0 || !A || !B || !Cm) return fail(nullptr, MRHWENO_ERR_INVALID_ARG, "bad GEMM arguments");
  MR_MLP_CHECK(mr_mlp_gemm((hipStream_t)stream, M, N, K, A, sAm, sAk, B, sBk, sBn, Cm, sCm, sCn));
  return MRHWENO_OK;
}

mrhweno_status mrhweno_mlp_forward(void* stream, const void* x, const void* params, void* cache, void* z, int batch) {
  if (!x || !params || !cache || !z || batch <= 0) return fail(nullptr, MRHWENO_ERR_INVALID_ARG, "bad forward arguments");
  MR_MLP_CHECK(mr_mlp_forward((hipStream_t)stream, x, params, cache, z, batch));
  return MRHWENO_OK;
}

mrhweno_status mrhweno_mlp_backward(void* stream, const void* x, const void* params, void* cache, const void* labels,
                                    void* grads, void* loss, int batch) {
  if (!x || !params || !cache || !labels || !grads || !loss || batch <= 0)
    return fail(nullptr, MRHWENO_ERR_INVALID_ARG, "bad backward arguments");
  MR_MLP_CHECK(mr_mlp_backward((hipStream_t)stream, x, params, cache, labels, grads, loss, batch));
  return MRHWENO_OK;
}

mrhweno_status mrhweno_mlp_adam(void* stream, void* master, void* params, const void* grads, void* m, void* v,
                                int step, float lr, float beta1, float beta2, float eps) {
  if (!master || !params || !grads || !m || !v || step < 1 || !(lr > 0.f) || !(beta1 >= 0.f && beta1 < 1.f) ||
      !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f))
    return fail(nullptr, MRHWENO_ERR_INVALID_ARG, "bad Adam arguments");
  MR_MLP_CHECK(mr_mlp_adam((hipStream_t)stream, master, params, grads, m, v, step, lr, beta1, beta2, eps));
  return MRHWENO_OK;
}

const char* mrhweno_last_error(const mrhweno_ctx* c) {
  if (c) return c->err.c_str();
  return g_err.c_str();
}

void mrhweno_destroy(mrhweno_ctx* c) {
  if (!c) return;
  if (c->exec) (void)hipGraphExecDestroy(c->exec);
  if (c->graph) (void)hipGraphDestroy(c->graph);
  delete c;
}

}  /* extern "C" */
