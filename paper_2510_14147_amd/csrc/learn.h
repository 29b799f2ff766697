// Learned cost model: shared declarations.
#pragma once

#include "tree.h"

namespace fnn {

constexpr int MLP_F = 16, MLP_H = 64, MLP_O = 2;
constexpr int MLP_NPAR = MLP_H * MLP_F + MLP_H + MLP_H * MLP_H + MLP_H +
                         MLP_O * MLP_H + MLP_O;  // 5378

struct FeatArgs {
    const int32_t *pack_of, *leaf_of, *parent, *depth, *center_pos, *pb, *pe,
        *ccnt, *q_cpos, *q_pb, *q_pe;
    const float *radius, *q_rad;
    float eps;
    // batch of clouds: per-cloud eps (CloudThr::feps) and the cloud of each
    // position, whose root is vertex 1 + cloud; null for a single cloud
    const CloudThr *ct;
    const int32_t *pcl;
    int first_pack, npacks;  // query-tree ids of the packs: first_pack + k
};

void tree_aux(fnn_tree *T, Scratch &S);
void compute_features(const fnn_tree *T, const Pts &P, float eps,
                      const CloudThr *ct, float *feat, hipStream_t s);
void mlp_forward(const float *theta, const float *X, long long n, float *Y,
                 hipStream_t s);
double mlp_loss_grad(const float *theta, const float *X, const float *T,
                     long long n, float *grad, Scratch &S);
// Allocation-free full-batch gradient: partial sums in a fixed device array
// (mlp_noalloc_scratch_bytes), grad and *loss (device) written in a fixed
// summation order.
void mlp_loss_grad_noalloc(const float *theta, const float *X, const float *T,
                           long long n, float *grad, double *loss, hipStream_t s);
size_t mlp_noalloc_scratch_bytes();
void mlp_train(float *theta, const float *X, const float *T, long long n,
               int epochs, int batch, float lr, unsigned long long seed,
               double *epoch_loss, Scratch &S);

}  // namespace fnn
