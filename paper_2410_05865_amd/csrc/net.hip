// Learned initial guess: a small 3D U-Net (BF16 activations and weights, FP32
// accumulation on MFMA) that maps (scaled right-hand side, geometry) on a grid
// to a scaled solution.  The multigrid solve still decides the result: the
// network only supplies phi_0.  Not part of the paper's method; an addition on top of it.
//
// Architecture (C = base channels, D = 3 or 4 levels, grid n divisible by
// 2^(D+1)); encoder channels w_l = C on the upper levels, 2C on the two coarsest:
//   e_0 = relu(conv(x, 16 -> w_0))                       n      (x: 2 input channels padded to 16)
//   e_l = relu(conv(pool(e_{l-1}), w_{l-1} -> w_l))      n/2^l, l = 1 .. D-2
//   b   = relu(conv(pool(e_{D-2}), w_{D-2} -> w_{D-1}))  n/2^(D-1)
//   d_l = relu(conv([up(d_{l+1}), e_l], w_{l+1} + w_l -> w_l))   l = D-2 .. 0 (d_{D-1} = b)
//   y   = conv(d_0, w_0 -> 16)[channel 0]                n      (output channels 1..15 held at 0)
// conv: 3x3x3, zero padding, bias; pool: 2x2x2 average; up: nearest.
// D = 3 with C = 32 has 521k parameters, D = 4 with C = 32 581k.
//
// Activations are channel-last ([batch][voxel][channel], voxel i + n (j + n k)).
// A conv is an implicit GEMM (voxels x taps*Cin x Cout): a wavefront computes
// 16 voxels x Cout, on v_mfma_f32_16x16x32_bf16 (gfx950's double-K BF16 MFMA,
// 32 input channels per instruction) where Cin is a multiple of 32, else on
// v_mfma_f32_16x16x16_bf16.  Backward: data gradients are the forward conv of
// the output gradient with the transposed, flipped kernel; weight gradients
// are a GEMM over voxels staged through LDS (32 voxels per MFMA), one
// workgroup per (tap, voxel range) writing per-range partials that a second
// kernel adds in a fixed order (no atomics: training is reproducible).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <memory>
#include <random>
#include <string>
#include <vector>

#include "common.hpp"

namespace cc {
namespace {

#define NETCHK(expr)                                                                           \
  do {                                                                                         \
    hipError_t _e = (expr);                                                                    \
    if (_e != hipSuccess) fail(CC_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(_e)); \
  } while (0)

typedef short v4s __attribute__((ext_vector_type(4)));
typedef short v8s __attribute__((ext_vector_type(8)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef float v4f __attribute__((ext_vector_type(4)));

// D (16 x 16) += A (16 x 32) B (32 x 16) in BF16: lane l holds A[l % 16][8 (l / 16) + t]
// and B[8 (l / 16) + t][l % 16], t = 0..7, and D[4 (l / 16) + q][l % 16], q = 0..3
__device__ __forceinline__ v4f mfma32(v8s a, v8s b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(v8bf, a), __builtin_bit_cast(v8bf, b), c, 0, 0,
                                                  0);
}

__host__ __device__ inline uint16_t f2bf(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest even
  return (uint16_t)(u >> 16);
}
__host__ __device__ inline float bf2f(uint16_t b) {
  uint32_t u = (uint32_t)b << 16;
  float f;
  std::memcpy(&f, &u, 4);
  return f;
}

// element (b, v, c) of a channel slice: p[(b * n3 + v) * cs + co + c]
struct View {
  uint16_t* p;
  int cs, co;
};

// ---------------------------------------------------------------- conv forward
// grid: nb * n^3 / 64 blocks of 256 threads (4 waves x 16 voxels).
template <int NT, bool K32>
__global__ void __launch_bounds__(256) k_conv_fwd(int n, View in, int cin, const uint16_t* __restrict__ wt,
                                                  const float* __restrict__ bias, int relu, View out,
                                                  float* __restrict__ out32) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const long long n3 = (long long)n * n * n;
  const long long vg0 = ((long long)blockIdx.x * 4 + wave) * 16;  // first voxel (global over the batch)
  const int r = lane & 15, kg = lane >> 4;
  const long long vg = vg0 + r;
  const long long b = vg / n3;
  const int v = (int)(vg - b * n3);
  const int i = v % n, j = (v / n) % n, k = v / (n * n);
  const int cout = NT * 16;
  v4f acc[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = v4f{0.f, 0.f, 0.f, 0.f};
  for (int tap = 0; tap < 27; ++tap) {
    const int dx = tap % 3 - 1, dy = (tap / 3) % 3 - 1, dz = tap / 9 - 1;
    const int ii = i + dx, jj = j + dy, kk = k + dz;
    const bool inside = ii >= 0 && ii < n && jj >= 0 && jj < n && kk >= 0 && kk < n;
    const long long vn = b * n3 + ii + (long long)n * (jj + (long long)n * kk);
    if constexpr (K32) {
      // 32 input channels per instruction: lane group kg holds channels 8 kg .. 8 kg + 7
      const uint16_t* arow = in.p + vn * in.cs + in.co + 8 * kg;
      const uint16_t* wrow = wt + ((long long)tap * cout + r) * cin + 8 * kg;
      for (int ci0 = 0; ci0 < cin; ci0 += 32) {
        v8s a = v8s{0, 0, 0, 0, 0, 0, 0, 0};
        if (inside) a = *reinterpret_cast<const v8s*>(arow + ci0);
#pragma unroll
        for (int t = 0; t < NT; ++t) {
          const v8s bw = *reinterpret_cast<const v8s*>(wrow + (long long)t * 16 * cin + ci0);
          acc[t] = mfma32(a, bw, acc[t]);
        }
      }
    } else {
      const uint16_t* arow = in.p + vn * in.cs + in.co + 4 * kg;
      const uint16_t* wrow = wt + ((long long)tap * cout + r) * cin + 4 * kg;
      for (int ci0 = 0; ci0 < cin; ci0 += 16) {
        v4s a = v4s{0, 0, 0, 0};
        if (inside) a = *reinterpret_cast<const v4s*>(arow + ci0);
#pragma unroll
        for (int t = 0; t < NT; ++t) {
          const v4s bw = *reinterpret_cast<const v4s*>(wrow + (long long)t * 16 * cin + ci0);
          acc[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, bw, acc[t], 0, 0, 0);
        }
      }
    }
  }
  // lane holds D[4 kg + q][r]: voxel vg0 + 4 kg + q, channel t * 16 + r
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int c = t * 16 + r;
    const float bs = bias ? bias[c] : 0.f;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const long long vo = vg0 + 4 * kg + q;
      float val = acc[t][q] + bs;
      if (relu) val = fmaxf(val, 0.f);
      out.p[vo * out.cs + out.co + c] = f2bf(val);
      if (out32 && c == 0) out32[vo] = val;
    }
  }
}

// ---------------------------------------------------------------- weight gradient
// part[split][tap][co][ci] = sum over the split's voxels of g[v][co] *
// in[v + off(tap)][ci]; k_sum_parts adds the splits in a fixed order (no
// atomics, so gradients and training are reproducible).
// grid (27, splits); 256 threads; voxels of the split staged 64 at a time in LDS.
constexpr int kWgChunk = 64;
__global__ void __launch_bounds__(256) k_conv_wgrad(int n, long long nvox, View in, int cin, View g, int cout,
                                                    float* __restrict__ part, long long per_split) {
  extern __shared__ uint16_t lds[];
  uint16_t* lg = lds;                        // [64][cout]
  uint16_t* li = lds + kWgChunk * cout;      // [64][cin]
  const int tap = blockIdx.x;
  const int dx = tap % 3 - 1, dy = (tap / 3) % 3 - 1, dz = tap / 9 - 1;
  const long long n3 = (long long)n * n * n;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r = lane & 15, kg = lane >> 4;
  const int tm = cout / 16, tn = cin / 16, ntile = tm * tn;
  // up to 8 tiles per wave (cout, cin <= 128 -> <= 64 tiles)
  v4f acc[8];
#pragma unroll
  for (int t = 0; t < 8; ++t) acc[t] = v4f{0.f, 0.f, 0.f, 0.f};
  const long long v_begin = (long long)blockIdx.y * per_split;
  const long long v_end = v_begin + per_split < nvox ? v_begin + per_split : nvox;
  for (long long c0 = v_begin; c0 < v_end; c0 += kWgChunk) {
    __syncthreads();
    for (int e = threadIdx.x; e < kWgChunk * cout; e += 256) {
      const int vv = e / cout, c = e % cout;
      const long long vg = c0 + vv;
      lg[e] = (vg < v_end) ? g.p[vg * g.cs + g.co + c] : (uint16_t)0;
    }
    for (int e = threadIdx.x; e < kWgChunk * cin; e += 256) {
      const int vv = e / cin, c = e % cin;
      const long long vg = c0 + vv;
      uint16_t val = 0;
      if (vg < v_end) {
        const long long b = vg / n3;
        const int v = (int)(vg - b * n3);
        const int ii = v % n + dx, jj = (v / n) % n + dy, kk = v / (n * n) + dz;
        if (ii >= 0 && ii < n && jj >= 0 && jj < n && kk >= 0 && kk < n)
          val = in.p[(b * n3 + ii + (long long)n * (jj + (long long)n * kk)) * in.cs + in.co + c];
      }
      li[e] = val;
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int tile = wave + 4 * t;
      if (tile >= ntile) break;
      const int m0 = (tile / tn) * 16, n0 = (tile % tn) * 16;
#pragma unroll
      for (int ks = 0; ks < kWgChunk; ks += 32) {
        v8s a, bw;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const int vv = ks + 8 * kg + q;
          a[q] = (short)lg[vv * cout + m0 + r];
          bw[q] = (short)li[vv * cin + n0 + r];
        }
        acc[t] = mfma32(a, bw, acc[t]);
      }
    }
  }
#pragma unroll
  for (int t = 0; t < 8; ++t) {
    const int tile = wave + 4 * t;
    if (tile >= ntile) break;
    const int m0 = (tile / tn) * 16, n0 = (tile % tn) * 16;
    float* out = part + (long long)blockIdx.y * 27 * cout * cin;
#pragma unroll
    for (int q = 0; q < 4; ++q) out[((long long)tap * cout + m0 + 4 * kg + q) * cin + n0 + r] = acc[t][q];
  }
}

// per-block bias-gradient partials part[block][c] (cout divides 256); the
// block's threads of one channel are added in thread order
__global__ void __launch_bounds__(256) k_bias_grad(long long nvox, View g, int cout, float* __restrict__ part) {
  __shared__ float sh[256];
  const int c = threadIdx.x % cout;
  const int lanes_per_c = blockDim.x / cout;
  float s = 0.f;
  for (long long v = (long long)blockIdx.x * lanes_per_c + threadIdx.x / cout; v < nvox;
       v += (long long)gridDim.x * lanes_per_c)
    s += bf2f(g.p[v * g.cs + g.co + c]);
  sh[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x < cout) {
    float t = 0.f;
    for (int k = 0; k < lanes_per_c; ++k) t += sh[threadIdx.x + k * cout];
    part[(long long)blockIdx.x * cout + threadIdx.x] = t;
  }
}

// out[e] = sum over s < nparts of part[s * count + e], s ascending
__global__ void k_sum_parts(long long count, int nparts, const float* __restrict__ part, float* __restrict__ out) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= count) return;
  float t = 0.f;
  for (int q = 0; q < nparts; ++q) t += part[(long long)q * count + e];
  out[e] = t;
}

// flipped transpose: wf[26 - tap][ci][co] = wt[tap][co][ci]
__global__ void k_flip(const uint16_t* __restrict__ wt, int cout, int cin, uint16_t* __restrict__ wf) {
  long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= 27LL * cout * cin) return;
  const int ci = (int)(e % cin), co = (int)((e / cin) % cout), tap = (int)(e / ((long long)cin * cout));
  wf[((long long)(26 - tap) * cin + ci) * cout + co] = wt[e];
}

// ---------------------------------------------------------------- pointwise
__global__ void k_pool(int n, int nb, View in, View out, int C) {
  // out at n/2
  const int m = n / 2;
  const long long m3 = (long long)m * m * m, n3 = (long long)n * n * n;
  long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nb * m3 * C) return;
  const int c = (int)(e % C);
  const long long vg = e / C, b = vg / m3;
  const int v = (int)(vg - b * m3);
  const int I = v % m, J = (v / m) % m, K = v / (m * m);
  float s = 0.f;
  for (int d = 0; d < 8; ++d) {
    const int i = 2 * I + (d & 1), j = 2 * J + ((d >> 1) & 1), k = 2 * K + (d >> 2);
    s += bf2f(in.p[(b * n3 + i + (long long)n * (j + (long long)n * k)) * in.cs + in.co + c]);
  }
  out.p[vg * out.cs + out.co + c] = f2bf(0.125f * s);
}
// gin (at n) += gout(parent) / 8
__global__ void k_pool_bwd_add(int n, int nb, View gout, View gin, int C) {
  const int m = n / 2;
  const long long m3 = (long long)m * m * m, n3 = (long long)n * n * n;
  long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nb * n3 * C) return;
  const int c = (int)(e % C);
  const long long vg = e / C, b = vg / n3;
  const int v = (int)(vg - b * n3);
  const int i = v % n, j = (v / n) % n, k = v / (n * n);
  const long long p = b * m3 + (i / 2) + (long long)m * ((j / 2) + (long long)m * (k / 2));
  uint16_t* dst = &gin.p[vg * gin.cs + gin.co + c];
  *dst = f2bf(bf2f(*dst) + 0.125f * bf2f(gout.p[p * gout.cs + gout.co + c]));
}
// out (at n) = in(parent at n/2)
__global__ void k_up(int n, int nb, View in, View out, int C) {
  const int m = n / 2;
  const long long m3 = (long long)m * m * m, n3 = (long long)n * n * n;
  long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nb * n3 * C) return;
  const int c = (int)(e % C);
  const long long vg = e / C, b = vg / n3;
  const int v = (int)(vg - b * n3);
  const int i = v % n, j = (v / n) % n, k = v / (n * n);
  const long long p = b * m3 + (i / 2) + (long long)m * ((j / 2) + (long long)m * (k / 2));
  out.p[vg * out.cs + out.co + c] = in.p[p * in.cs + in.co + c];
}
// gin (at n/2) = sum over the 8 children of gout (at n)
__global__ void k_up_bwd(int n, int nb, View gout, View gin, int C) {
  const int m = n / 2;
  const long long m3 = (long long)m * m * m, n3 = (long long)n * n * n;
  long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nb * m3 * C) return;
  const int c = (int)(e % C);
  const long long vg = e / C, b = vg / m3;
  const int v = (int)(vg - b * m3);
  const int I = v % m, J = (v / m) % m, K = v / (m * m);
  float s = 0.f;
  for (int d = 0; d < 8; ++d) {
    const int i = 2 * I + (d & 1), j = 2 * J + ((d >> 1) & 1), k = 2 * K + (d >> 2);
    s += bf2f(gout.p[(b * n3 + i + (long long)n * (j + (long long)n * k)) * gout.cs + gout.co + c]);
  }
  gin.p[vg * gin.cs + gin.co + c] = f2bf(s);
}
__global__ void k_relu_bwd(long long nvox, int C, View g, View y) {
  long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nvox * C) return;
  const int c = (int)(e % C);
  const long long v = e / C;
  if (!(bf2f(y.p[v * y.cs + y.co + c]) > 0.f)) g.p[v * g.cs + g.co + c] = 0;
}
// x (fp32 [voxel][2]) -> bf16 [voxel][16], channels 2..15 zero
__global__ void k_pack(long long nvox, const float* __restrict__ x, uint16_t* __restrict__ out) {
  long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nvox * 16) return;
  const int c = (int)(e % 16);
  const long long v = e / 16;
  out[e] = c < 2 ? f2bf(x[v * 2 + c]) : (uint16_t)0;
}
// masked mean-square loss on channel 0: per-block partial sums of (y - t)^2 and
// of the mask; gradient 2 (y - t) / count into g (bf16 [voxel][16], other
// channels 0).  count comes from a first pass (k_count).
// sum of a 256-thread block in a fixed order, valid in thread 0
__device__ __forceinline__ float block_sum256(float s) {
  __shared__ float w[4];
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  if ((threadIdx.x & 63) == 0) w[threadIdx.x >> 6] = s;
  __syncthreads();
  return (w[0] + w[1]) + (w[2] + w[3]);
}
__global__ void __launch_bounds__(256) k_count(long long nvox, const uint8_t* __restrict__ mask,
                                               float* __restrict__ part) {
  long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const float s = block_sum256((v < nvox && mask[v]) ? 1.f : 0.f);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}
__global__ void __launch_bounds__(256) k_loss(long long nvox, const float* __restrict__ y,
                                              const float* __restrict__ t, const uint8_t* __restrict__ mask,
                                              const float* __restrict__ count, float* __restrict__ part,
                                              uint16_t* __restrict__ g) {
  long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  float s = 0.f;
  if (v < nvox) {
    const float cnt = fmaxf(*count, 1.f);
    float d = mask[v] ? (y[v] - t[v]) : 0.f;
    s = d * d;
    if (g) {
      g[v * 16] = f2bf(2.f * d / cnt);
      for (int c = 1; c < 16; ++c) g[v * 16 + c] = 0;
    }
  }
  s = block_sum256(s);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}
__global__ void k_adam(long long np, float* __restrict__ w, const float* __restrict__ gr, float* __restrict__ m,
                       float* __restrict__ v2, float lr, float b1, float b2, float eps, float c1, float c2,
                       const uint8_t* __restrict__ frozen) {
  long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= np || frozen[e]) return;
  const float g = gr[e];
  m[e] = b1 * m[e] + (1.f - b1) * g;
  v2[e] = b2 * v2[e] + (1.f - b2) * g * g;
  w[e] -= lr * (m[e] / c1) / (sqrtf(v2[e] / c2) + eps);
}
__global__ void k_to_bf16(long long np, const float* __restrict__ w, uint16_t* __restrict__ o) {
  long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < np) o[e] = f2bf(w[e]);
}
__global__ void k_fill0(long long count, float* __restrict__ p) {
  long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < count) p[e] = 0.f;
}
__global__ void k_fill0_u16(long long count, uint16_t* __restrict__ p) {
  long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < count) p[e] = 0;
}

inline int nblk(long long count, int bs = 256) { return (int)((count + bs - 1) / bs); }

// ---------------------------------------------------------------- host side
struct Layer {
  int cin, cout;
  long long offW, offB;  // offsets into the flat FP32 parameter array
};

struct DevMem {
  std::vector<void*> ptrs;
  template <class T>
  T* alloc(size_t n) {
    void* p = nullptr;
    if (n == 0) n = 1;
    hipError_t e = hipMalloc(&p, n * sizeof(T));
    if (e != hipSuccess) fail(CC_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
    ptrs.push_back(p);
    return (T*)p;
  }
  void release() {
    for (void* p : ptrs) (void)hipFree(p);
    ptrs.clear();
  }
};

}  // namespace
}  // namespace cc

using namespace cc;

struct cc_net {
  int C = 16;
  int depth = 3;              // levels of the U-Net (3 or 4)
  hipStream_t stream = nullptr;
  std::vector<Layer> layers;  // encoder 0 .. depth-2, bottleneck, decoder depth-2 .. 0, output
  std::vector<int> width;     // channels of the encoder levels 0 .. depth-1
  long long np = 0;
  DevMem pmem;                // parameters and optimizer state
  float* w = nullptr;         // FP32 master weights
  float* g = nullptr;         // gradients
  float* m = nullptr;
  float* v = nullptr;
  uint8_t* frozen = nullptr;  // padded output channels stay 0
  uint16_t* wb = nullptr;     // BF16 copy
  uint16_t* wf = nullptr;     // flipped transpose scratch (largest layer)
  long long step = 0;
  // activations for (n, nb), per level l: CAT[l] = [up(coarser result) | e_l]
  // (the encoder output written beside the upsampled decoder input), P[l] the
  // pooled e_l, DD[l] the decoder output; BT the bottleneck
  int an = 0, anb = 0;
  DevMem amem;
  uint16_t *X0 = nullptr, *BT = nullptr, *Y = nullptr, *GY = nullptr, *GBT = nullptr;
  std::vector<uint16_t*> CAT, P, DD, GCAT, GP, GDD;
  float* Y32 = nullptr;
  float* red = nullptr;       // [0] loss sum, [1] mask count
  float* part = nullptr;      // per-split / per-block gradient and loss partials
};

namespace cc {
namespace {

template <bool K32>
void launch_conv_k(cc_net* N, int n, int nb, View in, int cin, const uint16_t* wt, const float* bias, int cout,
                   int relu, View out, float* out32) {
  const long long nvox = (long long)nb * n * n * n;
  dim3 grid((unsigned)(nvox / 64)), block(256);
  switch (cout / 16) {
    case 1: hipLaunchKernelGGL((k_conv_fwd<1, K32>), grid, block, 0, N->stream, n, in, cin, wt, bias, relu, out, out32); break;
    case 2: hipLaunchKernelGGL((k_conv_fwd<2, K32>), grid, block, 0, N->stream, n, in, cin, wt, bias, relu, out, out32); break;
    case 3: hipLaunchKernelGGL((k_conv_fwd<3, K32>), grid, block, 0, N->stream, n, in, cin, wt, bias, relu, out, out32); break;
    case 4: hipLaunchKernelGGL((k_conv_fwd<4, K32>), grid, block, 0, N->stream, n, in, cin, wt, bias, relu, out, out32); break;
    case 6: hipLaunchKernelGGL((k_conv_fwd<6, K32>), grid, block, 0, N->stream, n, in, cin, wt, bias, relu, out, out32); break;
    case 8: hipLaunchKernelGGL((k_conv_fwd<8, K32>), grid, block, 0, N->stream, n, in, cin, wt, bias, relu, out, out32); break;
    default: fail(CC_EINVAL, "unsupported channel count");
  }
}
// the double-K instruction where the input channels come in whole groups of 32
void launch_conv(cc_net* N, int n, int nb, View in, int cin, const uint16_t* wt, const float* bias, int cout,
                 int relu, View out, float* out32) {
  if (cin % 32 == 0)
    launch_conv_k<true>(N, n, nb, in, cin, wt, bias, cout, relu, out, out32);
  else
    launch_conv_k<false>(N, n, nb, in, cin, wt, bias, cout, relu, out, out32);
}

// gradients of one conv layer: dW, db from (in, g); gin = conv(g, flipped W) if gin.p
constexpr int kBiasBlocks = 256;
inline int wgrad_splits(long long nvox) { return (int)std::min<long long>(256, std::max<long long>(1, nvox / 4096)); }

void conv_backward(cc_net* N, const Layer& L, int n, int nb, View in, View g, View gin) {
  const long long nvox = (long long)nb * n * n * n;
  const int splits = wgrad_splits(nvox);
  const long long per = ((nvox + splits - 1) / splits + kWgChunk - 1) / kWgChunk * kWgChunk;
  const size_t lds = (size_t)kWgChunk * (L.cout + L.cin) * sizeof(uint16_t);
  const long long nw = 27LL * L.cout * L.cin;
  hipLaunchKernelGGL(k_conv_wgrad, dim3(27, splits), dim3(256), lds, N->stream, n, nvox, in, L.cin, g, L.cout,
                     N->part, per);
  hipLaunchKernelGGL(k_sum_parts, dim3(nblk(nw)), dim3(256), 0, N->stream, nw, splits, N->part, N->g + L.offW);
  hipLaunchKernelGGL(k_bias_grad, dim3(kBiasBlocks), dim3(256), 0, N->stream, nvox, g, L.cout, N->part);
  hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(256), 0, N->stream, (long long)L.cout, kBiasBlocks, N->part,
                     N->g + L.offB);
  if (gin.p) {
    const long long nw = 27LL * L.cout * L.cin;
    hipLaunchKernelGGL(k_flip, dim3(nblk(nw)), dim3(256), 0, N->stream, N->wb + L.offW, L.cout, L.cin, N->wf);
    launch_conv(N, n, nb, g, L.cout, N->wf, nullptr, L.cin, 0, gin, nullptr);
  }
}

// layer indices: encoder l (0 .. D-2), bottleneck D-1, decoder l at 2D-2-l, output 2D-1
inline int level_of_layer(int D, int li) {
  if (li < D - 1) return li;
  if (li == D - 1) return D - 1;
  if (li < 2 * D - 1) return 2 * D - 2 - li;
  return 0;
}

void ensure_acts(cc_net* N, int n, int nb) {
  if (N->an == n && N->anb == nb) return;
  N->amem.release();
  const int D = N->depth;
  const std::vector<int>& w = N->width;
  DevMem& A = N->amem;
  std::vector<long long> v(D);
  for (int l = 0; l < D; ++l) v[l] = ((long long)nb * n * n * n) >> (3 * l);
  N->X0 = A.alloc<uint16_t>(v[0] * 16);
  N->Y = A.alloc<uint16_t>(v[0] * 16);
  N->GY = A.alloc<uint16_t>(v[0] * 16);
  N->BT = A.alloc<uint16_t>(v[D - 1] * w[D - 1]);
  N->GBT = A.alloc<uint16_t>(v[D - 1] * w[D - 1]);
  N->CAT.assign(D - 1, nullptr);
  N->P.assign(D - 1, nullptr);
  N->DD.assign(D - 1, nullptr);
  N->GCAT.assign(D - 1, nullptr);
  N->GP.assign(D - 1, nullptr);
  N->GDD.assign(D - 1, nullptr);
  for (int l = 0; l < D - 1; ++l) {
    N->CAT[l] = A.alloc<uint16_t>(v[l] * (w[l + 1] + w[l]));
    N->GCAT[l] = A.alloc<uint16_t>(v[l] * (w[l + 1] + w[l]));
    N->P[l] = A.alloc<uint16_t>(v[l + 1] * w[l]);
    N->GP[l] = A.alloc<uint16_t>(v[l + 1] * w[l]);
    N->DD[l] = A.alloc<uint16_t>(v[l] * w[l]);
    N->GDD[l] = A.alloc<uint16_t>(v[l] * w[l]);
  }
  N->Y32 = A.alloc<float>(v[0]);
  N->red = A.alloc<float>(2);
  // partials: the largest of splits x 27 cout cin over the layers (at their
  // resolutions), the bias partials, and two per-block loss arrays
  {
    long long need = 2LL * nblk(v[0]);
    for (size_t li = 0; li < N->layers.size(); ++li) {
      const Layer& L = N->layers[li];
      const long long nv = v[level_of_layer(D, (int)li)];
      need = std::max(need, (long long)wgrad_splits(nv) * 27 * L.cout * L.cin);
      need = std::max(need, (long long)kBiasBlocks * L.cout);
    }
    N->part = A.alloc<float>((size_t)need);
  }
  N->an = n;
  N->anb = nb;
}

// views of level l: the concatenation, its upsampled part and its skip part
inline View cat_view(cc_net* N, int l) { return View{N->CAT[l], N->width[l + 1] + N->width[l], 0}; }
inline View skip_view(cc_net* N, int l) {
  return View{N->CAT[l], N->width[l + 1] + N->width[l], N->width[l + 1]};
}
inline View gcat_view(cc_net* N, int l) { return View{N->GCAT[l], N->width[l + 1] + N->width[l], 0}; }
inline View gskip_view(cc_net* N, int l) {
  return View{N->GCAT[l], N->width[l + 1] + N->width[l], N->width[l + 1]};
}

void forward(cc_net* N, int n, int nb, const float* x) {
  const int D = N->depth;
  const std::vector<int>& w = N->width;
  hipStream_t st = N->stream;
  const std::vector<Layer>& L = N->layers;
  const long long v0 = (long long)nb * n * n * n;
  hipLaunchKernelGGL(k_pack, dim3(nblk(v0 * 16)), dim3(256), 0, st, v0, x, N->X0);
  // encoder: conv + ReLU into the skip slot, then 2x2x2 average pooling
  View in{N->X0, 16, 0};
  int cin = 16;
  for (int l = 0; l < D - 1; ++l) {
    const int nl = n >> l;
    launch_conv(N, nl, nb, in, cin, N->wb + L[l].offW, N->w + L[l].offB, w[l], 1, skip_view(N, l), nullptr);
    const long long vn = ((long long)nb * nl * nl * nl) / 8;
    hipLaunchKernelGGL(k_pool, dim3(nblk(vn * w[l])), dim3(256), 0, st, nl, nb, skip_view(N, l), View{N->P[l], w[l], 0},
                       w[l]);
    in = View{N->P[l], w[l], 0};
    cin = w[l];
  }
  const int nc = n >> (D - 1);
  launch_conv(N, nc, nb, in, cin, N->wb + L[D - 1].offW, N->w + L[D - 1].offB, w[D - 1], 1, View{N->BT, w[D - 1], 0},
              nullptr);
  // decoder: nearest upsampling of the coarser result beside the skip, conv + ReLU
  View cur{N->BT, w[D - 1], 0};
  for (int l = D - 2; l >= 0; --l) {
    const int nl = n >> l;
    const long long vl = (long long)nb * nl * nl * nl;
    hipLaunchKernelGGL(k_up, dim3(nblk(vl * w[l + 1])), dim3(256), 0, st, nl, nb, cur, cat_view(N, l), w[l + 1]);
    const Layer& Ld = L[2 * D - 2 - l];
    launch_conv(N, nl, nb, cat_view(N, l), w[l + 1] + w[l], N->wb + Ld.offW, N->w + Ld.offB, w[l], 1,
                View{N->DD[l], w[l], 0}, nullptr);
    cur = View{N->DD[l], w[l], 0};
  }
  const Layer& Lo = L[2 * D - 1];
  launch_conv(N, n, nb, cur, w[0], N->wb + Lo.offW, N->w + Lo.offB, 16, 0, View{N->Y, 16, 0}, N->Y32);
}

void backward(cc_net* N, int n, int nb) {
  const int D = N->depth;
  const std::vector<int>& w = N->width;
  hipStream_t st = N->stream;
  const std::vector<Layer>& L = N->layers;
  const View none{nullptr, 0, 0};
  auto vox = [&](int l) { return ((long long)nb * n * n * n) >> (3 * l); };
  // output layer, then the decoder from the finest level down
  conv_backward(N, L[2 * D - 1], n, nb, View{N->DD[0], w[0], 0}, View{N->GY, 16, 0}, View{N->GDD[0], w[0], 0});
  hipLaunchKernelGGL(k_relu_bwd, dim3(nblk(vox(0) * w[0])), dim3(256), 0, st, vox(0), w[0], View{N->GDD[0], w[0], 0},
                     View{N->DD[0], w[0], 0});
  for (int l = 0; l < D - 1; ++l) {
    const int nl = n >> l;
    conv_backward(N, L[2 * D - 2 - l], nl, nb, cat_view(N, l), View{N->GDD[l], w[l], 0}, gcat_view(N, l));
    // the upsampled part's gradient, summed over each parent's 8 children
    const bool bott = l + 1 == D - 1;
    const View gnext = bott ? View{N->GBT, w[D - 1], 0} : View{N->GDD[l + 1], w[l + 1], 0};
    const View act = bott ? View{N->BT, w[D - 1], 0} : View{N->DD[l + 1], w[l + 1], 0};
    hipLaunchKernelGGL(k_up_bwd, dim3(nblk(vox(l + 1) * w[l + 1])), dim3(256), 0, st, nl, nb, gcat_view(N, l), gnext,
                       w[l + 1]);
    hipLaunchKernelGGL(k_relu_bwd, dim3(nblk(vox(l + 1) * w[l + 1])), dim3(256), 0, st, vox(l + 1), w[l + 1], gnext,
                       act);
  }
  // bottleneck, then the encoder from the coarsest level up
  conv_backward(N, L[D - 1], n >> (D - 1), nb, View{N->P[D - 2], w[D - 2], 0}, View{N->GBT, w[D - 1], 0},
                View{N->GP[D - 2], w[D - 2], 0});
  for (int l = D - 2; l >= 0; --l) {
    const int nl = n >> l;
    hipLaunchKernelGGL(k_pool_bwd_add, dim3(nblk(vox(l) * w[l])), dim3(256), 0, st, nl, nb, View{N->GP[l], w[l], 0},
                       gskip_view(N, l), w[l]);
    hipLaunchKernelGGL(k_relu_bwd, dim3(nblk(vox(l) * w[l])), dim3(256), 0, st, vox(l), w[l], gskip_view(N, l),
                       skip_view(N, l));
    const View in = l == 0 ? View{N->X0, 16, 0} : View{N->P[l - 1], w[l - 1], 0};
    const View gin = l == 0 ? none : View{N->GP[l - 1], w[l - 1], 0};
    conv_backward(N, L[l], nl, nb, in, gskip_view(N, l), gin);
  }
}

void check_shape(const cc_net* N, int n, int nb) {
  // the coarsest level (n / 2^(depth-1)) must hold whole 64-voxel groups per sample
  const int q = 4 << (N->depth - 1);
  if (n < q || n % q != 0)
    fail(CC_EINVAL, "grid size must be a positive multiple of " + std::to_string(q) + " for this depth");
  if (nb < 1) fail(CC_EINVAL, "batch must be positive");
}

template <class F>
int net_guard(F&& f) {
  try {
    f();
    return CC_OK;
  } catch (const Error& e) {
    set_last_error(e.what());
    return e.code;
  } catch (const std::bad_alloc&) {
    set_last_error("host allocation failed");
    return CC_ENOMEM;
  } catch (const std::exception& e) {
    set_last_error(e.what());
    return CC_EINVAL;
  }
}

}  // namespace
}  // namespace cc

extern "C" {

int cc_net_create(int base_channels, int depth, unsigned long long seed, void* stream, cc_net** out) {
  return net_guard([&] {
    if (!out) fail(CC_EINVAL, "null output");
    *out = nullptr;
    if (base_channels != 16 && base_channels != 32) fail(CC_EINVAL, "base_channels must be 16 or 32");
    if (depth != 3 && depth != 4) fail(CC_EINVAL, "depth must be 3 or 4");
    auto N = std::make_unique<cc_net>();
    N->C = base_channels;
    N->depth = depth;
    N->stream = (hipStream_t)stream;
    const int C = base_channels, D = depth;
    // encoder channels: C on the upper levels, 2C on the two coarsest
    for (int l = 0; l < D; ++l) N->width.push_back(l < D - 2 ? C : 2 * C);
    const std::vector<int>& wd = N->width;
    std::vector<std::pair<int, int>> io = {{16, wd[0]}};
    for (int l = 1; l < D - 1; ++l) io.push_back({wd[l - 1], wd[l]});
    io.push_back({wd[D - 2], wd[D - 1]});
    for (int l = D - 2; l >= 0; --l) io.push_back({wd[l + 1] + wd[l], wd[l]});
    io.push_back({wd[0], 16});
    long long off = 0;
    for (auto& p : io) {
      Layer L{p.first, p.second, off, off + 27LL * p.first * p.second};
      off = L.offB + p.second;
      N->layers.push_back(L);
    }
    N->np = off;
    // He-normal weights over the real fan-in; padded input (first layer,
    // channels 2..15) and output (last layer, channels 1..15) weights are 0 and
    // the latter frozen
    std::vector<float> w(off, 0.f);
    std::vector<uint8_t> frozen(off, 0);
    std::mt19937_64 rng(seed);
    const size_t last = N->layers.size() - 1;
    for (size_t li = 0; li < N->layers.size(); ++li) {
      const Layer& L = N->layers[li];
      const int real_in = li == 0 ? 2 : L.cin;
      std::normal_distribution<float> nd(0.f, std::sqrt(2.f / (27.f * real_in)));
      for (int tap = 0; tap < 27; ++tap)
        for (int co = 0; co < L.cout; ++co)
          for (int ci = 0; ci < L.cin; ++ci) {
            long long e = L.offW + ((long long)tap * L.cout + co) * L.cin + ci;
            bool pad = (li == 0 && ci >= 2) || (li == last && co >= 1);
            w[e] = pad ? 0.f : nd(rng);
            if (li == last && co >= 1) frozen[e] = 1;
          }
      for (int co = 0; co < L.cout; ++co)
        if (li == last && co >= 1) frozen[L.offB + co] = 1;
    }
    DevMem& P = N->pmem;
    N->w = P.alloc<float>(off);
    N->g = P.alloc<float>(off);
    N->m = P.alloc<float>(off);
    N->v = P.alloc<float>(off);
    N->frozen = P.alloc<uint8_t>(off);
    N->wb = P.alloc<uint16_t>(off);
    long long wmax = 0;
    for (const Layer& L : N->layers) wmax = std::max(wmax, 27LL * L.cin * L.cout);
    N->wf = P.alloc<uint16_t>(wmax);
    NETCHK(hipMemcpy(N->w, w.data(), off * sizeof(float), hipMemcpyHostToDevice));
    NETCHK(hipMemcpy(N->frozen, frozen.data(), off, hipMemcpyHostToDevice));
    hipLaunchKernelGGL(k_fill0, dim3(nblk(off)), dim3(256), 0, N->stream, off, N->g);
    hipLaunchKernelGGL(k_fill0, dim3(nblk(off)), dim3(256), 0, N->stream, off, N->m);
    hipLaunchKernelGGL(k_fill0, dim3(nblk(off)), dim3(256), 0, N->stream, off, N->v);
    hipLaunchKernelGGL(k_to_bf16, dim3(nblk(off)), dim3(256), 0, N->stream, off, N->w, N->wb);
    NETCHK(hipStreamSynchronize(N->stream));
    *out = N.release();
  });
}

long long cc_net_num_params(const cc_net* N) { return N ? N->np : 0; }

int cc_net_get_params(const cc_net* N, float* host) {
  return net_guard([&] {
    if (!N || !host) fail(CC_EINVAL, "null argument");
    NETCHK(hipMemcpyAsync(host, N->w, N->np * sizeof(float), hipMemcpyDeviceToHost, N->stream));
    NETCHK(hipStreamSynchronize(N->stream));
  });
}

int cc_net_set_params(cc_net* N, const float* host) {
  return net_guard([&] {
    if (!N || !host) fail(CC_EINVAL, "null argument");
    NETCHK(hipMemcpyAsync(N->w, host, N->np * sizeof(float), hipMemcpyHostToDevice, N->stream));
    hipLaunchKernelGGL(k_to_bf16, dim3(nblk(N->np)), dim3(256), 0, N->stream, N->np, N->w, N->wb);
    NETCHK(hipStreamSynchronize(N->stream));
  });
}

int cc_net_forward(cc_net* N, int n, int nb, const float* x, float* y) {
  return net_guard([&] {
    if (!N || !x || !y) fail(CC_EINVAL, "null argument");
    check_shape(N, n, nb);
    ensure_acts(N, n, nb);
    forward(N, n, nb, x);
    const long long v1 = (long long)nb * n * n * n;
    NETCHK(hipMemcpyAsync(y, N->Y32, v1 * sizeof(float), hipMemcpyDeviceToDevice, N->stream));
    NETCHK(hipStreamSynchronize(N->stream));
  });
}

int cc_net_loss_grad(cc_net* N, int n, int nb, const float* x, const float* target, const unsigned char* mask,
                     double* loss, float* grad_host) {
  return net_guard([&] {
    if (!N || !x || !target || !mask) fail(CC_EINVAL, "null argument");
    check_shape(N, n, nb);
    ensure_acts(N, n, nb);
    const long long v1 = (long long)nb * n * n * n;
    hipStream_t st = N->stream;
    forward(N, n, nb, x);
    const int nbk = nblk(v1);
    hipLaunchKernelGGL(k_count, dim3(nbk), dim3(256), 0, st, v1, mask, N->part);
    hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(64), 0, st, 1LL, nbk, N->part, N->red + 1);
    hipLaunchKernelGGL(k_loss, dim3(nbk), dim3(256), 0, st, v1, N->Y32, target, mask, N->red + 1, N->part + nbk,
                       N->GY);
    hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(64), 0, st, 1LL, nbk, N->part + nbk, N->red);
    // gradient buffers that are accumulated into must start at zero
    for (int l = 0; l < N->depth - 1; ++l) {
      const long long cnt = (v1 >> (3 * l)) * (N->width[l + 1] + N->width[l]);
      hipLaunchKernelGGL(k_fill0_u16, dim3(nblk(cnt)), dim3(256), 0, st, cnt, N->GCAT[l]);
    }
    hipLaunchKernelGGL(k_fill0, dim3(nblk(N->np)), dim3(256), 0, st, N->np, N->g);
    backward(N, n, nb);
    float red[2];
    NETCHK(hipMemcpyAsync(red, N->red, sizeof(red), hipMemcpyDeviceToHost, st));
    NETCHK(hipStreamSynchronize(st));
    if (loss) *loss = red[1] > 0 ? (double)red[0] / red[1] : 0.0;
    if (grad_host) {
      NETCHK(hipMemcpyAsync(grad_host, N->g, N->np * sizeof(float), hipMemcpyDeviceToHost, st));
      NETCHK(hipStreamSynchronize(st));
    }
  });
}

int cc_net_adam_step(cc_net* N, float lr, float beta1, float beta2, float eps) {
  return net_guard([&] {
    if (!N) fail(CC_EINVAL, "null argument");
    if (!(lr >= 0.f) || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f))
      fail(CC_EINVAL, "bad optimizer parameters");
    N->step += 1;
    const float c1 = 1.f - std::pow(beta1, (float)N->step), c2 = 1.f - std::pow(beta2, (float)N->step);
    hipLaunchKernelGGL(k_adam, dim3(nblk(N->np)), dim3(256), 0, N->stream, N->np, N->w, N->g, N->m, N->v, lr, beta1,
                       beta2, eps, c1, c2, N->frozen);
    hipLaunchKernelGGL(k_to_bf16, dim3(nblk(N->np)), dim3(256), 0, N->stream, N->np, N->w, N->wb);
    NETCHK(hipStreamSynchronize(N->stream));
  });
}

void cc_net_destroy(cc_net* N) {
  if (!N) return;
  if (N->stream) (void)hipStreamSynchronize(N->stream);
  N->amem.release();
  N->pmem.release();
  delete N;
}

}  // extern "C"
