/* Sizes and layouts of the learned troubled-cell indicator (2D Euler).
 *
 * Network 320 -> 64 -> 64 -> 1 (ReLU, ReLU, sigmoid) on the feature vector
 * of a cell (301 features, zero-padded to 320).  Parameter vector, BF16 for
 * the network and FP32 for the training master copy, in this order:
 *   W1 [64][320] (row = hidden unit, column = feature), b1 [64],
 *   W2 [64][64]  (row = output unit, column = input unit), b2 [64],
 *   W3 [64], b3, then 7 padding entries. */
#pragma once
#include <stdint.h>

#define MR_NF 301   /* features: 300 normalised moments + log2(h)/16       */
#define MR_KP 320   /* padded feature count: 10 contraction blocks of 32    */
#define MR_NH 64    /* hidden width                                          */
#define MR_OFF_W1 0
#define MR_OFF_B1 (MR_OFF_W1 + MR_NH * MR_KP)
#define MR_OFF_W2 (MR_OFF_B1 + MR_NH)
#define MR_OFF_B2 (MR_OFF_W2 + MR_NH * MR_NH)
#define MR_OFF_W3 (MR_OFF_B2 + MR_NH)
#define MR_OFF_B3 (MR_OFF_W3 + MR_NH)
#define MR_NPARAM (MR_OFF_B3 + 8)

/* Weights of the fused inference kernel in operand order: fragment
 * (kb, m, lane) is the 16-byte A operand of v_mfma_f32_16x16x32_bf16 that
 * lane `lane` supplies for output rows 16m..16m+15 and contraction block kb,
 * so the work group fills its LDS copy with one linear read. */
#define MR_FRAG1 (MR_KP / 32 * 4 * 64)   /* layer 1: 10 blocks x 4 row tiles */
#define MR_FRAG2 (MR_NH / 32 * 4 * 64)   /* layer 2: 2 blocks x 4 row tiles  */
struct mr_learn_w {
  uint4 w1[MR_FRAG1];
  uint4 w2[MR_FRAG2];
  float b1[MR_NH], b2[MR_NH], w3[MR_NH];
  float b3, pad[3];
};

/* One entry of the list of cells the network left undecided. */
struct mr_band {
  int inst, e;   /* instance, index into its extended flag plane */
};
