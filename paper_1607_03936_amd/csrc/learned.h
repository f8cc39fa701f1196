// Learned coarse correction: FP32 3D convolutional network on the node grid of the velocity
// multigrid level Q1 on N/2, with hand-written forward, backward and Adam kernels (a reading:
// the paper has no learned component).  Layout of every field: [sample][channel][z][y][x].
#pragma once

#include <cstddef>

#include "wb_internal.h"

namespace wb {

constexpr int NET_H = 16;        // hidden channels
constexpr int NET_LAYERS = 4;    // 4 -> H -> H -> H -> 3
constexpr float NET_SLOPE = 0.1f;

// Flat parameter blob: per layer W [Cout][Cin][27] (tap = dx + 3 dy + 9 dz multiplies the
// input at offset (dx-1, dy-1, dz-1)), then b [Cout].
size_t net_param_count();
size_t net_layer_offset(int layer);  // offset of W of `layer` in the blob
int net_cin(int layer);
int net_cout(int layer);

// Work buffers of one network evaluation with batch B on an M^3 grid.
struct NetWork {
  int M = 0, B = 0;
  float* z[NET_LAYERS] = {};   // pre-activations [B][Cout][M^3] (z[3] = output)
  float* g[2] = {};            // gradient ping-pong [B][H][M^3]
  float* wt = nullptr;         // transposed weights of all layers (blob layout)
  float* part = nullptr;       // per-block weight-gradient partials
  size_t part_len = 0;
  double* loss_part = nullptr; // loss reduction partials
};
size_t net_work_bytes(int M, int B);
void net_work_carve(NetWork& w, int M, int B, void* base);

// out = z[3] = N_theta(x), x [B][4][M^3].
void net_forward(hipStream_t st, const float* params, const float* x, NetWork& w);
// After net_forward on the same x: loss (1/B) sum w (o - t)^2 into *loss_dev (FP64, device) and
// the parameter gradient into grad.
void net_backward(hipStream_t st, const float* params, const float* x, const float* t,
                  const float* wgt, NetWork& w, float* grad, double* loss_dev);
// Adam with bias correction (step >= 1).
void net_adam(hipStream_t st, size_t n, float* params, const float* grad, float* m, float* v,
              int step, float lr);
// He-uniform initial weights from the counter-based splitmix64 generator, zero biases and a
// zero output layer.
void net_init(hipStream_t st, float* params, unsigned long long seed);

// Node feature of a Q1 level with N elements per direction: mean of log10 coef over each
// element's 8 Gauss points, averaged over the elements sharing the node, divided by 5.
void launch_node_feature(hipStream_t st, int N, const double* coef, float* feat, float* elem_tmp);

// Network input from the node feature and a residual r [3][M^3]: [feat, r / rho], with
// rho^2 = sumsq / (3 M^3) read from device memory.
template <typename T>
void launch_net_input(hipStream_t st, int M, int B, const float* feat, const T* r,
                      const double* sumsq, float* x);
// delta = rho o dinv on interior nodes, 0 on the boundary (Dirichlet).
template <typename T>
void launch_net_delta(hipStream_t st, int M, const float* o, const T* dinv, const double* sumsq,
                      T* delta);
// alpha = clip((r, A delta) / (A delta, A delta), 0, 2) from dots[0] = (r, A delta),
// dots[1] = (A delta, A delta); x += alpha delta; counters[0] += (alpha > 0), counters[1] += !.
template <typename T>
void launch_net_guarded_update(hipStream_t st, size_t len, const double* dots, T* x,
                               const T* delta, int* counters);
// Training pair from an error e and its residual r = A e at a Q1 level: x = [feat, r / rho],
// t = d e / rho, w = rho^2 / (d sum_j d_j e_j^2) (t = w = 0 on the boundary), d = 1 / dinv;
// sums[0] = sum r^2, sums[1] = sum_interior e^2 / dinv.
void launch_net_pair(hipStream_t st, int M, const float* feat, const double* e, const double* r,
                     const double* dinv, const double* sums, float* x, float* t, float* w);
// sum over interior nodes of e_i^2 / dinv_i into *out (two-stage, deterministic).
void launch_energy_diag(hipStream_t st, int M, const double* e, const double* dinv,
                        double* partial, double* out);
// out[i] = 2 U(splitmix64(seed * 2^32 + i)) - 1 on interior nodes of a 3-component Q1 field,
// 0 on the boundary.
void launch_splitmix_field(hipStream_t st, int M, unsigned long long seed, double* out);

}  // namespace wb
