// HIP kernels (gfx950) of the learned coarse correction: 3x3x3 convolutions (forward, the
// adjoint in the input, weight gradients), loss, Adam, the node feature, training pairs and the
// guarded correction step.  FP32 network arithmetic; the reductions accumulate in FP64.
#include <algorithm>
#include <cmath>
#include <vector>

#include "learned.h"

namespace wb {

namespace {

constexpr int TX = 8, TY = 8, TZ = 4, TN = TX * TY * TZ;      // 256 nodes per block
constexpr int HX = TX + 2, HY = TY + 2, HZ = TZ + 2, HN = HX * HY * HZ;  // tile with halo

inline unsigned grid1(size_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }
inline int ntiles(int M) {
  return ((M + TX - 1) / TX) * ((M + TY - 1) / TY) * ((M + TZ - 1) / TZ);
}

__device__ __forceinline__ float leaky(float v) { return v > 0.f ? v : NET_SLOPE * v; }

struct TileIdx {
  int x0, y0, z0;
};
__device__ inline TileIdx tile_of(int M) {
  const int nx = (M + TX - 1) / TX, ny = (M + TY - 1) / TY;
  const int t = blockIdx.x;
  TileIdx r;
  r.x0 = (t % nx) * TX;
  r.y0 = ((t / nx) % ny) * TY;
  r.z0 = (t / (nx * ny)) * TZ;
  return r;
}

// C channels of the input tile with a one-node halo into LDS (zero outside the grid),
// optionally through the leaky ReLU.
template <int C, bool ACT>
__device__ inline void load_halo(const float* __restrict__ in, int M, size_t M3, const TileIdx& ti,
                                 float* s) {
  for (int idx = threadIdx.x; idx < C * HN; idx += TN) {
    const int c = idx / HN, h = idx - c * HN;
    const int hx = h % HX, hy = (h / HX) % HY, hz = h / (HX * HY);
    const int gx = ti.x0 + hx - 1, gy = ti.y0 + hy - 1, gz = ti.z0 + hz - 1;
    float v = 0.f;
    if (gx >= 0 && gx < M && gy >= 0 && gy < M && gz >= 0 && gz < M) {
      v = in[(size_t)c * M3 + gx + (size_t)M * (gy + (size_t)M * gz)];
      if (ACT) v = leaky(v);
    }
    s[idx] = v;
  }
}

// 3x3x3 convolution with zero padding, one output node per thread, all CO channels.
// MODE bit 0: leaky ReLU applied to the input on load; bit 1: output multiplied by
// leaky'(zmul) (the adjoint through the previous activation).  Weight addresses are uniform
// over the block (scalar loads); the input tile sits in LDS.
template <int CI, int CO, int MODE>
__global__ void __launch_bounds__(TN)
k_conv(int M, const float* __restrict__ in, const float* __restrict__ w,
       const float* __restrict__ bias, const float* __restrict__ zmul, float* __restrict__ out) {
  __shared__ float s[CI * HN];
  const size_t M3 = (size_t)M * M * M;
  const int b = blockIdx.y;
  const TileIdx ti = tile_of(M);
  load_halo<CI, (MODE & 1) != 0>(in + (size_t)b * CI * M3, M, M3, ti, s);
  __syncthreads();
  const int t = threadIdx.x;
  const int lx = t % TX, ly = (t / TX) % TY, lz = t / (TX * TY);
  float acc[CO];
#pragma unroll
  for (int co = 0; co < CO; ++co) acc[co] = bias != nullptr ? bias[co] : 0.f;
  for (int ci = 0; ci < CI; ++ci) {
    const float* sc = s + ci * HN + lx + HX * (ly + HY * lz);
#pragma unroll
    for (int tap = 0; tap < 27; ++tap) {
      const float v = sc[(tap % 3) + HX * ((tap / 3) % 3 + HY * (tap / 9))];
#pragma unroll
      for (int co = 0; co < CO; ++co) acc[co] += w[(co * CI + ci) * 27 + tap] * v;
    }
  }
  const int gx = ti.x0 + lx, gy = ti.y0 + ly, gz = ti.z0 + lz;
  if (gx < M && gy < M && gz < M) {
    const size_t g = gx + (size_t)M * (gy + (size_t)M * gz);
#pragma unroll
    for (int co = 0; co < CO; ++co) {
      float o = acc[co];
      if (MODE & 2) o *= zmul[((size_t)b * CO + co) * M3 + g] > 0.f ? 1.f : NET_SLOPE;
      out[((size_t)b * CO + co) * M3 + g] = o;
    }
  }
}

// Weight-gradient partials of one block (one tile of one sample):
// dW[co][ci][tap] = sum_nodes gz[co][n] a[ci][n + offset(tap)], db[co] = sum_nodes gz[co][n],
// a = leaky(in) when ACT.  Thread t handles the pair p = t % P over the nodes t / P + k G.
template <int CI, int CO, bool ACT>
__global__ void __launch_bounds__(TN)
k_wgrad(int M, const float* __restrict__ in, const float* __restrict__ gz, float* __restrict__ part) {
  constexpr int P = CI * CO;
  static_assert(P <= TN, "one thread per weight pair at least");
  constexpr int G = TN / P;
  constexpr int SH = CI * HN + CO * TN, RED = G * P * 28;
  __shared__ float sh[SH > RED ? SH : RED];
  float* s = sh;
  float* gs = sh + CI * HN;
  const size_t M3 = (size_t)M * M * M;
  const int b = blockIdx.y;
  const TileIdx ti = tile_of(M);
  load_halo<CI, ACT>(in + (size_t)b * CI * M3, M, M3, ti, s);
  for (int idx = threadIdx.x; idx < CO * TN; idx += TN) {
    const int co = idx / TN, node = idx - co * TN;
    const int gx = ti.x0 + node % TX, gy = ti.y0 + (node / TX) % TY, gz_ = ti.z0 + node / (TX * TY);
    float v = 0.f;
    if (gx < M && gy < M && gz_ < M)
      v = gz[((size_t)b * CO + co) * M3 + gx + (size_t)M * (gy + (size_t)M * gz_)];
    gs[idx] = v;
  }
  __syncthreads();
  const int t = threadIdx.x;
  float acc[28];
#pragma unroll
  for (int j = 0; j < 28; ++j) acc[j] = 0.f;
  if (t < G * P) {
    const int p = t % P, grp = t / P, co = p / CI, ci = p % CI;
    const float* sc = s + ci * HN;
    for (int node = grp; node < TN; node += G) {
      const float gv = gs[co * TN + node];
      const float* sn = sc + node % TX + HX * ((node / TX) % TY + HY * (node / (TX * TY)));
#pragma unroll
      for (int tap = 0; tap < 27; ++tap)
        acc[tap] += gv * sn[(tap % 3) + HX * ((tap / 3) % 3 + HY * (tap / 9))];
      acc[27] += gv;
    }
  }
  __syncthreads();
  if (t < G * P)
#pragma unroll
    for (int j = 0; j < 28; ++j) sh[t * 28 + j] = acc[j];
  __syncthreads();
  float* pb = part + (size_t)(blockIdx.y * gridDim.x + blockIdx.x) * (P * 27 + CO);
  for (int idx = t; idx < P * 27; idx += TN) {
    const int p = idx / 27, tap = idx - p * 27;
    float sum = 0.f;
    for (int g = 0; g < G; ++g) sum += sh[(g * P + p) * 28 + tap];
    pb[idx] = sum;  // p = co CI + ci: the blob layout of W
  }
  for (int co = t; co < CO; co += TN) {
    float sum = 0.f;
    for (int g = 0; g < G; ++g) sum += sh[(g * P + co * CI) * 28 + 27];  // ci = 0 lanes only
    pb[P * 27 + co] = sum;
  }
}

// grad[j] = sum over blocks of part[blk][j], fixed order.
__global__ void k_part_sum(int nblk, int len, const float* __restrict__ part, float* __restrict__ grad) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= len) return;
  double s = 0.0;
  for (int b = 0; b < nblk; ++b) s += part[(size_t)b * len + j];
  grad[j] = (float)s;
}

// transposed weights of a layer: wt[(ci CO + co) 27 + 26 - tap] = w[(co CI + ci) 27 + tap]
__global__ void k_transpose_w(int CI, int CO, const float* __restrict__ w, float* __restrict__ wt) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= CI * CO * 27) return;
  const int tap = j % 27, p = j / 27, ci = p % CI, co = p / CI;
  wt[(ci * CO + co) * 27 + 26 - tap] = w[j];
}

__device__ inline double block_sum_d(double v) {
  __shared__ double red[4];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) s = red[0] + red[1] + red[2] + red[3];
  __syncthreads();
  return s;
}

constexpr int NRED = 512;

// go = 2 w (o - t) / B and partial sums of w (o - t)^2 / B
__global__ void __launch_bounds__(256)
k_loss(size_t n, float invB, const float* __restrict__ o, const float* __restrict__ t,
       const float* __restrict__ w, float* __restrict__ go, double* __restrict__ partial) {
  double s = 0.0;
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
    const float d = o[i] - t[i];
    s += (double)w[i] * d * d;
    go[i] = 2.f * w[i] * d * invB;
  }
  s = block_sum_d(s);
  if (threadIdx.x == 0) partial[blockIdx.x] = s * invB;
}

__global__ void __launch_bounds__(256) k_sum_partials(int nb, const double* __restrict__ p, double* out) {
  double s = 0.0;
  for (int i = threadIdx.x; i < nb; i += 256) s += p[i];
  s = block_sum_d(s);
  if (threadIdx.x == 0) *out = s;
}

__global__ void k_adam(size_t n, float* __restrict__ p, const float* __restrict__ g,
                       float* __restrict__ m, float* __restrict__ v, float lr, float c1, float c2) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = 0.9f * m[i] + 0.1f * gi;
  const float vi = 0.999f * v[i] + 0.001f * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + 1e-8f);
}

__global__ void k_elem_logmean(int E, const double* __restrict__ coef, float* __restrict__ em) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= E) return;
  double s = 0.0;
  for (int q = 0; q < 8; ++q) s += log10(coef[(size_t)e * 8 + q]);
  em[e] = (float)(s / 8.0);
}

__global__ void k_node_feat(int N, const float* __restrict__ em, float* __restrict__ feat) {
  const int M = N + 1;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= M * M * M) return;
  const int x = i % M, y = (i / M) % M, z = i / (M * M);
  float s = 0.f;
  int c = 0;
  for (int ez = z - 1; ez <= z; ++ez)
    for (int ey = y - 1; ey <= y; ++ey)
      for (int ex = x - 1; ex <= x; ++ex)
        if (ex >= 0 && ex < N && ey >= 0 && ey < N && ez >= 0 && ez < N) {
          s += em[ex + N * (ey + N * ez)];
          ++c;
        }
  feat[i] = s / (float)c / 5.f;
}

__device__ inline bool on_boundary(int i, int M) {
  const int x = i % M, y = (i / M) % M, z = i / (M * M);
  return x == 0 || x == M - 1 || y == 0 || y == M - 1 || z == 0 || z == M - 1;
}

template <typename T>
__global__ void k_net_input(int M, const float* __restrict__ feat, const T* __restrict__ r,
                            const double* __restrict__ sumsq, float* __restrict__ x) {
  const int M3 = M * M * M;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= M3) return;
  const double rho = sqrt(*sumsq / (3.0 * M3));
  const double inv = rho > 0.0 ? 1.0 / rho : 0.0;
  x[i] = feat[i];
#pragma unroll
  for (int c = 0; c < 3; ++c) x[(size_t)(1 + c) * M3 + i] = (float)((double)r[(size_t)c * M3 + i] * inv);
}

template <typename T>
__global__ void k_net_delta(int M, const float* __restrict__ o, const T* __restrict__ dinv,
                            const double* __restrict__ sumsq, T* __restrict__ delta) {
  const int M3 = M * M * M;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= M3) return;
  const double rho = sqrt(*sumsq / (3.0 * M3));
  const bool bnd = on_boundary(i, M);
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const size_t j = (size_t)c * M3 + i;
    delta[j] = bnd ? T(0) : (T)(rho * (double)o[j] * (double)dinv[j]);
  }
}

// one thread: alpha from the two dot products, counters; alpha stored in dots[2]
__global__ void k_net_alpha(double* __restrict__ dots, int* __restrict__ counters) {
  const double num = dots[0], den = dots[1];
  double a = (den > 0.0 && isfinite(num) && isfinite(den)) ? num / den : 0.0;
  a = a < 0.0 ? 0.0 : (a > 2.0 ? 2.0 : a);
  dots[2] = a;
  if (a > 0.0) counters[0] += 1;
  else counters[1] += 1;
}

template <typename T>
__global__ void k_axpy_alpha(size_t n, const double* __restrict__ dots, T* __restrict__ x,
                             const T* __restrict__ delta) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const T a = (T)dots[2];
  x[i] += a * delta[i];
}

__global__ void k_net_pair(int M, const float* __restrict__ feat, const double* __restrict__ e,
                           const double* __restrict__ r, const double* __restrict__ dinv,
                           const double* __restrict__ sums, float* __restrict__ x,
                           float* __restrict__ t, float* __restrict__ w) {
  const int M3 = M * M * M;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= M3) return;
  const double rho = sqrt(sums[0] / (3.0 * M3));
  const double inv = rho > 0.0 ? 1.0 / rho : 0.0;
  const double en = sums[1];
  const bool bnd = on_boundary(i, M);
  x[i] = feat[i];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const size_t j = (size_t)c * M3 + i;
    x[(size_t)M3 + j] = (float)(r[j] * inv);
    if (bnd || !(en > 0.0)) {
      t[j] = 0.f;
      w[j] = 0.f;
    } else {
      const double d = 1.0 / dinv[j];
      t[j] = (float)(d * e[j] * inv);
      w[j] = (float)(rho * rho / (d * en));
    }
  }
}

__global__ void __launch_bounds__(256)
k_energy_diag(int M, const double* __restrict__ e, const double* __restrict__ dinv,
              double* __restrict__ partial) {
  const size_t M3 = (size_t)M * M * M, n = 3 * M3;
  double s = 0.0;
  for (size_t j = (size_t)blockIdx.x * 256 + threadIdx.x; j < n; j += (size_t)gridDim.x * 256)
    if (!on_boundary((int)(j % M3), M)) s += e[j] * e[j] / dinv[j];
  s = block_sum_d(s);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

__global__ void k_splitmix_field(int M, unsigned long long seed, double* __restrict__ out) {
  const size_t M3 = (size_t)M * M * M;
  const size_t j = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= 3 * M3) return;
  unsigned long long z = (seed << 32) + (unsigned long long)j + 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  z = z ^ (z >> 31);
  const double u = 2.0 * ((double)(z >> 11) * (1.0 / 9007199254740992.0)) - 1.0;
  out[j] = on_boundary((int)(j % M3), M) ? 0.0 : u;
}

}  // namespace

// ------------------------------------------------------------------ host side
int net_cin(int layer) { return layer == 0 ? 4 : NET_H; }
int net_cout(int layer) { return layer == NET_LAYERS - 1 ? 3 : NET_H; }
size_t net_layer_offset(int layer) {
  size_t o = 0;
  for (int l = 0; l < layer; ++l) o += (size_t)net_cout(l) * net_cin(l) * 27 + net_cout(l);
  return o;
}
size_t net_param_count() { return net_layer_offset(NET_LAYERS); }

namespace {
size_t part_len_max(int M, int B) {
  size_t mx = 0;
  for (int l = 0; l < NET_LAYERS; ++l)
    mx = std::max(mx, (size_t)ntiles(M) * B * ((size_t)net_cin(l) * net_cout(l) * 27 + net_cout(l)));
  return mx;
}
size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }
}  // namespace

size_t net_work_bytes(int M, int B) {
  const size_t M3 = (size_t)M * M * M;
  size_t b = 0;
  b += 3 * align256(sizeof(float) * B * NET_H * M3);   // z0..z2
  b += align256(sizeof(float) * B * 3 * M3);           // z3
  b += 2 * align256(sizeof(float) * B * NET_H * M3);   // g0, g1
  b += align256(sizeof(float) * net_param_count());    // wt
  b += align256(sizeof(float) * part_len_max(M, B));   // part
  b += align256(sizeof(double) * NRED);                // loss partials
  return b;
}

void net_work_carve(NetWork& w, int M, int B, void* base) {
  const size_t M3 = (size_t)M * M * M;
  char* p = static_cast<char*>(base);
  auto take = [&](size_t bytes) {
    char* q = p;
    p += align256(bytes);
    return q;
  };
  w.M = M;
  w.B = B;
  for (int l = 0; l < 3; ++l) w.z[l] = reinterpret_cast<float*>(take(sizeof(float) * B * NET_H * M3));
  w.z[3] = reinterpret_cast<float*>(take(sizeof(float) * B * 3 * M3));
  w.g[0] = reinterpret_cast<float*>(take(sizeof(float) * B * NET_H * M3));
  w.g[1] = reinterpret_cast<float*>(take(sizeof(float) * B * NET_H * M3));
  w.wt = reinterpret_cast<float*>(take(sizeof(float) * net_param_count()));
  w.part_len = part_len_max(M, B);
  w.part = reinterpret_cast<float*>(take(sizeof(float) * w.part_len));
  w.loss_part = reinterpret_cast<double*>(take(sizeof(double) * NRED));
}

void net_forward(hipStream_t st, const float* params, const float* x, NetWork& w) {
  const dim3 grid(ntiles(w.M), w.B);
  const float* W0 = params + net_layer_offset(0);
  const float* W1 = params + net_layer_offset(1);
  const float* W2 = params + net_layer_offset(2);
  const float* W3 = params + net_layer_offset(3);
  hipLaunchKernelGGL((k_conv<4, NET_H, 0>), grid, dim3(TN), 0, st, w.M, x, W0, W0 + NET_H * 4 * 27,
                     nullptr, w.z[0]);
  hipLaunchKernelGGL((k_conv<NET_H, NET_H, 1>), grid, dim3(TN), 0, st, w.M, w.z[0], W1,
                     W1 + NET_H * NET_H * 27, nullptr, w.z[1]);
  hipLaunchKernelGGL((k_conv<NET_H, NET_H, 1>), grid, dim3(TN), 0, st, w.M, w.z[1], W2,
                     W2 + NET_H * NET_H * 27, nullptr, w.z[2]);
  hipLaunchKernelGGL((k_conv<NET_H, 3, 1>), grid, dim3(TN), 0, st, w.M, w.z[2], W3,
                     W3 + 3 * NET_H * 27, nullptr, w.z[3]);
}

namespace {
template <int CI, int CO, bool ACT>
void wgrad(hipStream_t st, NetWork& w, int layer, const float* in, const float* gz, float* grad) {
  const dim3 grid(ntiles(w.M), w.B);
  hipLaunchKernelGGL((k_wgrad<CI, CO, ACT>), grid, dim3(TN), 0, st, w.M, in, gz, w.part);
  const int len = CI * CO * 27 + CO;
  hipLaunchKernelGGL(k_part_sum, dim3(grid1(len, 256)), dim3(256), 0, st, (int)(grid.x * grid.y),
                     len, w.part, grad + net_layer_offset(layer));
}
}  // namespace

void net_backward(hipStream_t st, const float* params, const float* x, const float* t,
                  const float* wgt, NetWork& w, float* grad, double* loss_dev) {
  const size_t M3 = (size_t)w.M * w.M * w.M;
  const size_t nout = (size_t)w.B * 3 * M3;
  const int nb = (int)std::min<size_t>(NRED, grid1(nout, 256));
  float* go = w.g[0];
  hipLaunchKernelGGL(k_loss, dim3(nb), dim3(256), 0, st, nout, 1.f / w.B, w.z[3], t, wgt, go,
                     w.loss_part);
  hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, st, nb, w.loss_part, loss_dev);
  for (int l = 1; l < NET_LAYERS; ++l) {
    const int n = net_cin(l) * net_cout(l) * 27;
    hipLaunchKernelGGL(k_transpose_w, dim3(grid1(n, 256)), dim3(256), 0, st, net_cin(l), net_cout(l),
                       params + net_layer_offset(l), w.wt + net_layer_offset(l));
  }
  const dim3 grid(ntiles(w.M), w.B);
  // layer 3 (H -> 3): input leaky(z2)
  wgrad<NET_H, 3, true>(st, w, 3, w.z[2], go, grad);
  hipLaunchKernelGGL((k_conv<3, NET_H, 2>), grid, dim3(TN), 0, st, w.M, go, w.wt + net_layer_offset(3),
                     nullptr, w.z[2], w.g[1]);
  // layer 2
  wgrad<NET_H, NET_H, true>(st, w, 2, w.z[1], w.g[1], grad);
  hipLaunchKernelGGL((k_conv<NET_H, NET_H, 2>), grid, dim3(TN), 0, st, w.M, w.g[1],
                     w.wt + net_layer_offset(2), nullptr, w.z[1], w.g[0]);
  // layer 1
  wgrad<NET_H, NET_H, true>(st, w, 1, w.z[0], w.g[0], grad);
  hipLaunchKernelGGL((k_conv<NET_H, NET_H, 2>), grid, dim3(TN), 0, st, w.M, w.g[0],
                     w.wt + net_layer_offset(1), nullptr, w.z[0], w.g[1]);
  // layer 0: input x as is
  wgrad<4, NET_H, false>(st, w, 0, x, w.g[1], grad);
}

void net_adam(hipStream_t st, size_t n, float* params, const float* grad, float* m, float* v,
              int step, float lr) {
  const double c1 = 1.0 / (1.0 - std::pow(0.9, step));
  const double c2 = 1.0 / (1.0 - std::pow(0.999, step));
  hipLaunchKernelGGL(k_adam, dim3(grid1(n, 256)), dim3(256), 0, st, n, params, grad, m, v, lr,
                     (float)c1, (float)c2);
}

void net_init(hipStream_t st, float* params, unsigned long long seed) {
  std::vector<float> h(net_param_count(), 0.f);
  size_t o = 0;
  unsigned long long ctr = 0;
  for (int l = 0; l < NET_LAYERS; ++l) {
    const int ci = net_cin(l), co = net_cout(l);
    // the output layer starts at zero: the untrained correction is delta = 0 (the plain
    // V-cycle, loss 1), and training moves away from it
    const double lim = l == NET_LAYERS - 1 ? 0.0 : std::sqrt(6.0 / (ci * 27.0));
    for (int j = 0; j < co * ci * 27; ++j, ++ctr) {
      unsigned long long z = (seed << 32) + ctr + 0x9E3779B97F4A7C15ULL;
      z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
      z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
      z = z ^ (z >> 31);
      h[o + j] = (float)(lim * (2.0 * ((double)(z >> 11) * (1.0 / 9007199254740992.0)) - 1.0));
    }
    o += (size_t)co * ci * 27 + co;
  }
  WB_HIP(hipMemcpyAsync(params, h.data(), sizeof(float) * h.size(), hipMemcpyHostToDevice, st));
  WB_HIP(hipStreamSynchronize(st));
}

void launch_node_feature(hipStream_t st, int N, const double* coef, float* feat, float* elem_tmp) {
  const int E = N * N * N, M = N + 1;
  hipLaunchKernelGGL(k_elem_logmean, dim3(grid1(E, 256)), dim3(256), 0, st, E, coef, elem_tmp);
  hipLaunchKernelGGL(k_node_feat, dim3(grid1((size_t)M * M * M, 256)), dim3(256), 0, st, N, elem_tmp,
                     feat);
}

template <typename T>
void launch_net_input(hipStream_t st, int M, int B, const float* feat, const T* r,
                      const double* sumsq, float* x) {
  (void)B;
  hipLaunchKernelGGL((k_net_input<T>), dim3(grid1((size_t)M * M * M, 256)), dim3(256), 0, st, M,
                     feat, r, sumsq, x);
}
template void launch_net_input<double>(hipStream_t, int, int, const float*, const double*,
                                       const double*, float*);
template void launch_net_input<float>(hipStream_t, int, int, const float*, const float*,
                                      const double*, float*);

template <typename T>
void launch_net_delta(hipStream_t st, int M, const float* o, const T* dinv, const double* sumsq,
                      T* delta) {
  hipLaunchKernelGGL((k_net_delta<T>), dim3(grid1((size_t)M * M * M, 256)), dim3(256), 0, st, M, o,
                     dinv, sumsq, delta);
}
template void launch_net_delta<double>(hipStream_t, int, const float*, const double*, const double*,
                                       double*);
template void launch_net_delta<float>(hipStream_t, int, const float*, const float*, const double*,
                                      float*);

template <typename T>
void launch_net_guarded_update(hipStream_t st, size_t len, const double* dots, T* x,
                               const T* delta, int* counters) {
  hipLaunchKernelGGL(k_net_alpha, dim3(1), dim3(1), 0, st, const_cast<double*>(dots), counters);
  hipLaunchKernelGGL((k_axpy_alpha<T>), dim3(grid1(len, 256)), dim3(256), 0, st, len, dots, x, delta);
}
template void launch_net_guarded_update<double>(hipStream_t, size_t, const double*, double*,
                                                const double*, int*);
template void launch_net_guarded_update<float>(hipStream_t, size_t, const double*, float*,
                                               const float*, int*);

void launch_net_pair(hipStream_t st, int M, const float* feat, const double* e, const double* r,
                     const double* dinv, const double* sums, float* x, float* t, float* w) {
  hipLaunchKernelGGL(k_net_pair, dim3(grid1((size_t)M * M * M, 256)), dim3(256), 0, st, M, feat, e,
                     r, dinv, sums, x, t, w);
}

void launch_energy_diag(hipStream_t st, int M, const double* e, const double* dinv,
                        double* partial, double* out) {
  const size_t n = (size_t)3 * M * M * M;
  const int nb = (int)std::min<size_t>(NRED, grid1(n, 256));
  hipLaunchKernelGGL(k_energy_diag, dim3(nb), dim3(256), 0, st, M, e, dinv, partial);
  hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, st, nb, partial, out);
}

void launch_splitmix_field(hipStream_t st, int M, unsigned long long seed, double* out) {
  const size_t n = (size_t)3 * M * M * M;
  hipLaunchKernelGGL(k_splitmix_field, dim3(grid1(n, 256)), dim3(256), 0, st, M, seed, out);
}

}  // namespace wb
