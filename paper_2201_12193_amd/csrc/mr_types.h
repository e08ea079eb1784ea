/* Shared host/device descriptors of the MR-HWENO GPU library.
 *
 * One mr_inst per problem instance lives in device memory (carved out of the
 * caller's workspace).  Its static part is written by the host at create
 * time; its dynamic part (time, step, state rotation, reductions, error
 * word) is advanced by the device so that a whole SSP-RK3 step runs without
 * a host round trip.
 */
#pragma once
#include <stdint.h>

#define MR_MAX_NC 4

/* Constants of the nonlinear weights (eqs. linear-weight, p, pq) derived on
 * the host from the user's positive linear weights gbar_1..4. */
struct mr_wconst {
  double g4[4];     /* gamma_{l,4} = gbar_l / S_4                              */
  double sg[4];     /* S_l / gbar_l, S_l = gbar_1 + ... + gbar_l               */
  double sgn[3];    /* S_l / gbar_{l+1}                                        */
  double eps;       /* epsilon of eqs. (w1_-LR), (non-linear-weight)          */
};

struct mr_inst {
  /* ---- static ---- */
  int dim, nx, ny, nc;
  int flux;         /* 0 = Burgers + Lax-Friedrichs, 1 = Euler + HLLC          */
  int bcx, bcy;     /* fold kinds of the low (bits 0-1) and high (bits 2-3) side:
                       0 = periodic, 1 = transmissive (also inflow sides, whose
                       ghosts are then overwritten), 2 = reflective wall      */
  int pres;         /* bit s: side s (0 left, 1 right, 2 bottom, 3 top) has
                       ghosts that hold a prescribed state                     */
  int skind[4];     /* side kinds: 1 transmissive, 2 reflective, 3 inflow      */
  int stepi, stepj; /* 2D: a solid step of the cells i >= stepi, j < stepj
                       (stepj = 0: none); read as ghosts, mirror images      */
  int wallflux;     /* 1: exact mirror-problem flux on wall faces            */
  int tc;           /* 0 none, 1 KXRCF, 2 all cells, 3 learned, 4 TVB minmod    */
  int beta_on;      /* 0 = q_l, 1 = p_l                                        */
  int charwise;     /* 1D Euler: Step 1 on characteristic fields               */
  int mod;          /* where modified first moments go: 0 stage inputs and U^n,
                       1 nowhere (internal to L), 2 stage inputs only         */
  int fhalo, shalo; /* halo widths of the flag and summary planes              */
  int fex, fey;     /* flag plane extents                                      */
  int sex, sey;     /* summary plane extents                                   */
  long long plane;  /* nx * ny                                                 */
  double dx, dy, gam, cfl, t_final;
  double rdx, rdy;            /* 1/dx, 1/dy                                    */
  double band_lo, band_hi;  /* learned-indicator uncertainty band              */
  double tvb_mh2;           /* M h^2 of the TVB indicator                      */
  double x0, y0;            /* lower-left corner of the domain                 */
  double sstate[4][4];      /* inflow state of each side                       */
  double spre[4][4];        /* state of the ghosts before a side's front       */
  double ssplit[4][3];      /* front s0 + st t + sn nu (bottom and top)        */
  mr_wconst W;
  double* buf[3];             /* state rotation; buf[0] = caller's moments     */
  unsigned char* flags[2];    /* [0] stage-1 flags, [1] stage-2/3 flags        */
  double* summ;               /* KXRCF face summaries (extended planes)        */
  double* aleph;              /* optional KXRCF numerator/denominator output   */
  double* unm;                /* 2D: first moments of U^n after Step 2.2 of
                                 stage 1, [comp][2][ny][nx] (written by stage 1,
                                 read by the RK combination of stages 2, 3)   */
  /* ---- dynamic (device) ---- */
  double t, dt, t_prev;
  long long steps;
  int cur;                    /* buf index holding U^n                         */
  int active;                 /* current step advances the state               */
  int err;                    /* sticky non-physical / non-finite state flag   */
  int rolled;                 /* state rolled back to the last good step       */
  unsigned long long amax[2]; /* max wave speeds of U^n (IEEE bits, >= 0)      */
  unsigned long long lfa[3];  /* Lax-Friedrichs alpha of each stage input      */
  const double* p_in[3];      /* stage inputs of the current step              */
  double* p_out[3];           /* stage outputs                                 */
  const double* p_un;         /* U^n of the current step                       */
};

/* Work item of the 2D stage kernel: a column strip of one instance. */
struct mr_tile2 {
  int inst, x0, y0, rows;
};
/* Work item of the 1D stage kernel and of per-cell kernels. */
struct mr_tile1 {
  int inst, start, count, pad;
};
