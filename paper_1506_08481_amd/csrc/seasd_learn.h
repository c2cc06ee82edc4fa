// seasd_learn.h - internal interface of the learned preconditioner network
// (seasd_learn.hip) used by the solve and the training entry points.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/seasd.h"
#include "seasd_internal.h"

namespace seasd {

constexpr double kEdgeCut = 2.0;     // edges: |r| < 2 (a_i + a_j)
constexpr float kAgg = 1.0f / 16.0f; // message sum scale

// graph, edge and node features of the binned configuration held in A
int net_build_graph(seasd_net net, const ApplyArgs& A, hipStream_t st);
// forward pass over the current graph
int net_forward(seasd_net net, hipStream_t st);
// initial guess x0 for nrhs right-hand sides (gin == NULL), or, given gin =
// dL/dx0, the output gradients for net_backward ([nrhs][n][12] arrays)
int net_x0(seasd_net net, const double* inv, const int* perm, int nrhs, const double* b, const double* gin,
           double* x0, hipStream_t st);
int net_backward(seasd_net net, hipStream_t st);
int net_adam(seasd_net net, float lr, hipStream_t st);
// rescaled blocks S B S into out; *bad |= 1 on non-finite or extreme output
int net_learned_blocks(seasd_net net, const double* inv, const int* perm, double* out, int* bad, hipStream_t st);
int check_finite(int64_t len, const double* x, int* bad, hipStream_t st);
int net_grads_to_host(seasd_net net, float* host, int64_t count, hipStream_t st);
int net_device(seasd_net net);
int64_t net_edges(seasd_net net);

}  // namespace seasd
