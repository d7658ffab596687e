// Launch wrappers of the learned proposal's kernels (internal).
#pragma once
#include "round.hpp"

namespace pamo {

constexpr int LEARN_NFEAT = 32;    // features per edge (the first LEARN_NF_USED used)
constexpr int LEARN_NF_USED = 11;
constexpr int LEARN_NPARAM = 6337;  // W1 64x32 | b1 64 | W2 64x64 | b2 64 | W3 64 | b3
constexpr int MLP_O_W1 = 0, MLP_O_B1 = 2048, MLP_O_W2 = 2112, MLP_O_B2 = 6208, MLP_O_W3 = 6272, MLP_O_B3 = 6336;

// the network as the inference kernel reads it
struct MlpDev {
  __bf16 w1[64 * 32];  // [unit][input]
  __bf16 w2[64 * 64];
  float w3[64];
  float b1[64], b2[64];
  float b3;
  int a1, a2;
  float threshold;
};

// weight grids and activation shifts of a network being trained
struct MlpMeta {
  int e1, e2, e3, a1, a2;
};

// features of cand[0..*ncand) (bound >= *ncand sizes the grid) into X [n][32];
// with fmesh and use_m set, the rows of meshes with use_m[mesh] == 0 are zero
void launch_features(hipStream_t s, MeshView m, const uint64_t* key, const int* cand, const int* ncand, int bound,
                     const int* ovl, float* X, int* err, const int* fmesh = nullptr,
                     const uint8_t* use_m = nullptr);
// logits of X[0..*n_dev) into out (may be null); with key non-null, rows under
// the threshold set their edge cand[row] aside (largest key on both
// half-edges) and count into *ndemote (and ndemote_m[mesh] when fmesh is set;
// then only meshes with use_m[mesh] set candidates aside); with dlist set,
// the set-aside half-edges go to dlist[0..*ndemote) in no particular order
void launch_mlp(hipStream_t s, const float* X, const int* n_dev, int bound, const MlpDev* M, float* out,
                const int* cand, const int* twin, uint64_t* key, int* ndemote, const int* fmesh = nullptr,
                int* ndemote_m = nullptr, const uint8_t* use_m = nullptr, int* dlist = nullptr);
// batches: reason 5 (no flag) for the candidates of meshes that set
// candidates aside and committed nothing (their round runs again)
void launch_mark_retry(hipStream_t s, const int* cand, const int* ncand, int bound, const int* fmesh,
                       const int* demote_m, const int* commits_m, uint8_t* reason, const int* gate = nullptr);
// one batch of nb samples (rows order[base + i], or base + i when order is
// null; rows outside [0, nrows) are left out): per-block gradient sums into
// part [blocks][LEARN_NPARAM] and losses
void launch_train_grad(hipStream_t s, const float* P, MlpMeta meta, const float* X, const uint8_t* Y,
                       const int* order, int64_t base, int nb, int64_t nrows, float* part, float* part_loss);
// reduce the block sums; grad (may be null) gets the gradient; with am/av
// non-null an Adam step number t (>= 1) updates P
void launch_train_reduce(hipStream_t s, const float* part, const float* part_loss, int nb, MlpMeta meta, float* P,
                         float* grad, float* am, float* av, float lr, int64_t t, float* loss_out);
int train_blocks(int nb);
// append the rows of the candidates the checks decided (reason <= 3), in
// candidate order: features from Xs, label 1 when committed; at most room
// rows; *nrows = rows available this round
// reserve the row logger's buffers for up to `bound` candidates per round
void learn_reserve(Workspace& ws, int64_t bound);
void launch_log_rows(Workspace& ws, hipStream_t s, const int* ncand, int bound, const uint8_t* reason, const float* Xs,
                     float* X, uint8_t* y, int64_t room, int* nrows);
// distance of each point of P to the closest triangle of (V, F); the largest
// one is folded into *dmax_bits (the bits of a non-negative double, start 0)
void launch_point_surface(hipStream_t s, const double* P, int np, const double* V, const int* F, int nf,
                          double* dist, uint64_t* dmax_bits);

}  // namespace pamo
