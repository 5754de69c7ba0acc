// Device kernels of the multigrid solve (Sec. 5.3) for gfx950: the cell-averaged
// fourth-order stencil with wall ghosts (Sec. 2.3) used by SMO-1, residuals and
// restriction, piecewise-constant prolongation, FV-PLG rows, the level-by-level
// supernodal triangular solves of the LU-correction and bottom solver, max-norm
// reductions and right-hand-side cell averages.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "kernels.hpp"
#include "quadrature.hpp"

namespace cc {

namespace {

constexpr int kWave = 64;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, kWave));
  return v;
}

// One axis of the assembled regular row (times 12 h^2): the 5-point
// fourth-order stencil, with the ghost-substituted forms in the two cell layers
// next to a Dirichlet (bc 0) or Neumann (bc 1) wall.  Adds the diagonal to diag.
__device__ __forceinline__ double axis_op(const double* __restrict__ x, long c, long s, int t, int n,
                                          int blo, int bhi, double& diag) {
  if (t >= 2 && t <= n - 3) {
    diag += -30.0;
    return -x[c - 2 * s] + 16.0 * x[c - s] - 30.0 * x[c] + 16.0 * x[c + s] - x[c + 2 * s];
  }
  if (t == n - 1) {
    if (bhi == 0) {
      diag += -1087.0 / 12.0;
      return (21.0 * x[c - 3 * s] - 139.0 * x[c - 2 * s] + 545.0 * x[c - s] - 1087.0 * x[c]) / 12.0;
    }
    diag += -14.5;
    return 0.1 * x[c - 3 * s] - 1.5 * x[c - 2 * s] + 15.9 * x[c - s] - 14.5 * x[c];
  }
  if (t == n - 2) {
    if (bhi == 0) {
      diag += -403.0 / 12.0;
      return (-15.0 * x[c - 2 * s] + 209.0 * x[c - s] - 403.0 * x[c] + 269.0 * x[c + s]) / 12.0;
    }
    diag += -30.9;
    return -1.1 * x[c - 2 * s] + 16.5 * x[c - s] - 30.9 * x[c] + 15.5 * x[c + s];
  }
  if (t == 0) {
    if (blo == 0) {
      diag += -1087.0 / 12.0;
      return (21.0 * x[c + 3 * s] - 139.0 * x[c + 2 * s] + 545.0 * x[c + s] - 1087.0 * x[c]) / 12.0;
    }
    diag += -14.5;
    return 0.1 * x[c + 3 * s] - 1.5 * x[c + 2 * s] + 15.9 * x[c + s] - 14.5 * x[c];
  }
  // t == 1
  if (blo == 0) {
    diag += -403.0 / 12.0;
    return (-15.0 * x[c + 2 * s] + 209.0 * x[c + s] - 403.0 * x[c] + 269.0 * x[c - s]) / 12.0;
  }
  diag += -30.9;
  return -1.1 * x[c + 2 * s] + 16.5 * x[c + s] - 30.9 * x[c] + 15.5 * x[c - s];
}

// (L x)_c * 12 h^2 for a phi_1 cell and its diagonal.
__device__ __forceinline__ double regular_row(const StencilLevel& L, const double* __restrict__ x, int i,
                                              int j, int k, long c, double& diag) {
  const int n = L.n;
  const long nn = (long)n * n;
  diag = 0.0;
  double a = axis_op(x, c, 1, i, n, L.bc[0], L.bc[1], diag);
  a += axis_op(x, c, n, j, n, L.bc[2], L.bc[3], diag);
  a += axis_op(x, c, nn, k, n, L.bc[4], L.bc[5], diag);
  return a;
}

// 1D grid over 64 x 4 x 1 cell tiles, z fastest: concurrently resident blocks
// work on a narrow range of (x, y) columns, so the +-2 z-neighbour planes are
// re-read from cache (measured faster than x- or y-fastest orders).
__device__ __forceinline__ void tile_ijk(int n, int& i, int& j, int& k) {
  const int b = blockIdx.x;
  k = b % n;
  const int r = b / n;
  const int ny = (n + 3) / 4;
  j = (r % ny) * 4 + threadIdx.y;
  i = (r / ny) * 64 + threadIdx.x;
}

__global__ void k_smo1(StencilLevel L, double omega, const double* __restrict__ s, const double* __restrict__ ein,
                       double* __restrict__ eout) {
  const int n = L.n;
  int i, j, k;
  tile_ijk(n, i, j, k);
  if (i >= n || j >= n) return;
  long c = i + (long)n * (j + (long)n * k);
  double v = ein[c];
  if (L.type[c] == 1) {
    double diag;
    double a = regular_row(L, ein, i, j, k, c, diag);
    v += omega * (s[c] - a * L.inv12h2) / (diag * L.inv12h2);
  }
  eout[c] = v;
}

__global__ void k_stencil_residual(StencilLevel L, const double* __restrict__ r, const double* __restrict__ x,
                                   double* __restrict__ s, int apply) {
  const int n = L.n;
  int i, j, k;
  tile_ijk(n, i, j, k);
  if (i >= n || j >= n) return;
  long c = i + (long)n * (j + (long)n * k);
  double v = 0.0;
  if (L.type[c] == 1) {
    double diag;
    double a = regular_row(L, x, i, j, k, c, diag) * L.inv12h2;
    v = apply ? a : r[c] - a;
  }
  s[c] = v;
}

__global__ void k_plg_residual(PlgRows P, const double* __restrict__ r, const double* __restrict__ x,
                               double* __restrict__ s, int apply) {
  int row = blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= P.N2) return;
  double a = 0.0;
#pragma unroll 5
  for (int t = 0; t < 35; ++t) a += P.vals[(long)t * P.N2 + row] * x[P.cols[(long)t * P.N2 + row]];
  int c = P.cell[row];
  s[c] = apply ? a : r[c] - a;
}

__global__ void k_plg_b2(PlgRows P, const double* __restrict__ s, const double* __restrict__ e,
                         double* __restrict__ y) {
  int row = blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= P.N2) return;
  uint64_t m = P.phi2[row];
  double a = 0.0;
  for (int t = 0; t < 35; ++t)
    if (!((m >> t) & 1ull)) a += P.vals[(long)t * P.N2 + row] * e[P.cols[(long)t * P.N2 + row]];
  y[P.nd[row]] = s[P.cell[row]] - a;
}

// coarse cell = 2^-3 sum over its 8 children of (s - L e) on phi_1 children
__global__ void k_restrict(StencilLevel F, StencilLevel C, const double* __restrict__ s,
                           const double* __restrict__ e, double* __restrict__ sc) {
  const int nc = C.n, nf = F.n;
  int I, J, K;
  tile_ijk(nc, I, J, K);
  if (I >= nc || J >= nc) return;
  long cc = I + (long)nc * (J + (long)nc * K);
  double acc = 0.0;
  if (C.type[cc] != 0) {
    for (int dz = 0; dz < 2; ++dz)
      for (int dy = 0; dy < 2; ++dy)
        for (int dx = 0; dx < 2; ++dx) {
          int i = 2 * I + dx, j = 2 * J + dy, k = 2 * K + dz;
          long c = i + (long)nf * (j + (long)nf * k);
          if (F.type[c] != 1) continue;
          double diag;
          acc += s[c] - regular_row(F, e, i, j, k, c, diag) * F.inv12h2;
        }
  }
  sc[cc] = 0.125 * acc;
}

__global__ void k_prolong_add(StencilLevel F, int nc, const double* __restrict__ ec, double* __restrict__ ef) {
  const int n = F.n;
  int i, j, k;
  tile_ijk(n, i, j, k);
  if (i >= n || j >= n) return;
  long c = i + (long)n * (j + (long)n * k);
  if (F.type[c] == 1) ef[c] += ec[(i >> 1) + (long)nc * ((j >> 1) + (long)nc * (k >> 1))];
}

__global__ void k_gather(int n, const int* __restrict__ var_cell, const double* __restrict__ src,
                         double* __restrict__ y) {
  int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v < n) y[v] = src[var_cell[v]];
}

// Supernodal sweeps.  Rows of every node are stored row-major; the node's
// equations are numbered in pivot order, so its right-hand side is contiguous.
// A task is one wavefront handling 64/g rows of one node with g lanes per row:
// (node, first row, log2 g).

// acc += sum_{j in [j0, j1), j = gl mod g} a[j] * b[j], four independent chains
__device__ __forceinline__ double lane_dot(const double* __restrict__ a, const double* __restrict__ b, int j0,
                                           int j1, int gl, int g) {
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  int j = j0 + gl;
  for (; j + 3 * g < j1; j += 4 * g) {
    s0 += a[j] * b[j];
    s1 += a[j + g] * b[j + g];
    s2 += a[j + 2 * g] * b[j + 2 * g];
    s3 += a[j + 3 * g] * b[j + 3 * g];
  }
  for (; j < j1; j += g) s0 += a[j] * b[j];
  return (s0 + s1) + (s2 + s3);
}

// Forward sweep of one height: z_F = L11^-1 y_F on the node's rows, and
// y_U -= (L21 L11^-1) y_F accumulated atomically into the later equations.
__global__ void k_lu_forward(LuDev F, const LuTask* __restrict__ tasks, int ntasks) {
  int wave = (blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  int lane = threadIdx.x % kWave;
  if (wave >= ntasks) return;
  const LuTask t = tasks[wave];
  const int lg = t.lg, g = 1 << lg;
  const int sub = lane >> lg, gl = lane & (g - 1);
  const int p = t.p, q = t.q, base = t.base;
  const int i = t.row0 + sub;
  const bool valid = i < p + q;
  const double* yF = F.y + base;
  double acc = 0.0;
  if (valid) {
    if (i < p)
      acc = lane_dot(F.M + t.offM + (long)i * p, yF, 0, i, gl, g);
    else
      acc = lane_dot(F.V + t.offVW + (long)(i - p) * p, yF, 0, p, gl, g);
  }
  for (int o = g >> 1; o > 0; o >>= 1) acc += __shfl_xor(acc, o, kWave);
  if (valid && gl == 0) {
    if (i < p)
      F.z[base + i] = acc + yF[i];
    else
      atomicAdd(&F.y[F.Uf[t.offU + (i - p)]], -acc);
  }
}

// Backward sweep of one height: x_F = U11^-1 z_F - (U11^-1 U12) x_U, scattered
// to the grid array `out` through var_cell.
__global__ void k_lu_backward(LuDev F, const LuTask* __restrict__ tasks, int ntasks, double* __restrict__ out) {
  int wave = (blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  int lane = threadIdx.x % kWave;
  if (wave >= ntasks) return;
  const LuTask t = tasks[wave];
  const int lg = t.lg, g = 1 << lg;
  const int sub = lane >> lg, gl = lane & (g - 1);
  const int p = t.p, q = t.q, base = t.base;
  const int i = t.row0 + sub;
  const bool valid = i < p;
  double acc = 0.0;
  if (valid) {
    acc = lane_dot(F.M + t.offM + (long)i * p, F.z + base, i, p, gl, g);
    if (q > 0) {
      const double* Wr = F.W + t.offVW + (long)i * q;
      const int* U = F.U + t.offU;
      double s0 = 0.0, s1 = 0.0;
      int j = gl;
      for (; j + g < q; j += 2 * g) {
        s0 += Wr[j] * F.x[U[j]];
        s1 += Wr[j + g] * F.x[U[j + g]];
      }
      for (; j < q; j += g) s0 += Wr[j] * F.x[U[j]];
      acc -= s0 + s1;
    }
  }
  for (int o = g >> 1; o > 0; o >>= 1) acc += __shfl_xor(acc, o, kWave);
  if (valid && gl == 0) {
    F.x[base + i] = acc;
    out[F.var_cell[base + i]] = acc;
  }
}

__global__ void k_zero(double* p, long long count) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  long long stride = (long long)gridDim.x * blockDim.x;
  for (; i < count; i += stride) p[i] = 0.0;
}

__global__ void k_zero_u64(unsigned long long* p) { *p = 0ull; }

__global__ void k_maxabs(const double* __restrict__ v, long long count, unsigned long long* out) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  long long stride = (long long)gridDim.x * blockDim.x;
  double m = 0.0;
  for (; i < count; i += stride) m = fmax(m, fabs(v[i]));
  m = wave_max(m);
  if (threadIdx.x % kWave == 0) atomicMax(out, (unsigned long long)__double_as_longlong(m));
}

__global__ void k_add_unknowns(StencilLevel L, const double* __restrict__ e, double* __restrict__ phi) {
  long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  long long n3 = (long long)L.n * L.n * L.n;
  if (c < n3 && L.type[c] != 0) phi[c] += e[c];
}

__global__ void k_mask_unknowns(StencilLevel L, double* __restrict__ a) {
  long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  long long n3 = (long long)L.n * L.n * L.n;
  if (c < n3 && L.type[c] == 0) a[c] = 0.0;
}

__global__ void k_copy_pairs(int count, const int2* __restrict__ pairs, double* __restrict__ a) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < count) a[pairs[t].x] = a[pairs[t].y];
}

__global__ void k_set_values(int count, const int* __restrict__ cells, const double* __restrict__ vals,
                             double* __restrict__ a) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < count) a[cells[t]] = vals[t];
}

struct GaussQ {
  int q;
  double x[16], w[16];
};

__global__ void k_cell_average(int n, double h, double ox, double oy, double oz, FieldDesc f, int mode,
                               GaussQ G, double* __restrict__ out) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  int j = blockIdx.y * blockDim.y + threadIdx.y;
  int k = blockIdx.z;
  if (i >= n || j >= n) return;
  double cx = ox + (i + 0.5) * h, cy = oy + (j + 0.5) * h, cz = oz + (k + 0.5) * h;
  double acc = 0.0;
  for (int a = 0; a < G.q; ++a) {
    double z = cz + 0.5 * h * G.x[a];
    double sy = 0.0;
    for (int b = 0; b < G.q; ++b) {
      double y = cy + 0.5 * h * G.x[b];
      double sx = 0.0;
      for (int c = 0; c < G.q; ++c) sx += G.w[c] * field_value(f, cx + 0.5 * h * G.x[c], y, z, mode);
      sy += G.w[b] * sx;
    }
    acc += G.w[a] * sy;
  }
  out[i + (long)n * (j + (long)n * k)] = 0.125 * acc;
}

inline dim3 grid3(int n) { return dim3((n + 63) / 64, (n + 3) / 4, n); }
inline dim3 grid_tiles(int n) { return dim3(((n + 63) / 64) * ((n + 3) / 4) * n); }
const dim3 kBlock3(64, 4, 1);
inline int blocks(long long count, int bs) { return (int)((count + bs - 1) / bs); }

}  // namespace

void launch_smo1(const StencilLevel& L, double omega, const double* s, const double* e_in, double* e_out,
                 hipStream_t st) {
  hipLaunchKernelGGL(k_smo1, grid_tiles(L.n), kBlock3, 0, st, L, omega, s, e_in, e_out);
}
void launch_stencil_residual(const StencilLevel& L, const double* r, const double* x, double* s, hipStream_t st) {
  hipLaunchKernelGGL(k_stencil_residual, grid_tiles(L.n), kBlock3, 0, st, L, r, x, s, 0);
}
void launch_stencil_apply(const StencilLevel& L, const double* x, double* y, hipStream_t st) {
  hipLaunchKernelGGL(k_stencil_residual, grid_tiles(L.n), kBlock3, 0, st, L, (const double*)nullptr, x, y, 1);
}
void launch_plg_residual(const PlgRows& P, const double* r, const double* x, double* s, int apply_only,
                         hipStream_t st) {
  if (P.N2 == 0) return;
  hipLaunchKernelGGL(k_plg_residual, dim3(blocks(P.N2, 256)), dim3(256), 0, st, P, r, x, s, apply_only);
}
void launch_restrict(const StencilLevel& F, const StencilLevel& C, const double* s, const double* e, double* sc,
                     hipStream_t st) {
  hipLaunchKernelGGL(k_restrict, grid_tiles(C.n), kBlock3, 0, st, F, C, s, e, sc);
}
void launch_prolong_add(const StencilLevel& F, int nc, const double* ec, double* ef, hipStream_t st) {
  hipLaunchKernelGGL(k_prolong_add, grid_tiles(F.n), kBlock3, 0, st, F, nc, ec, ef);
}
void launch_plg_b2(const PlgRows& P, const double* s, const double* e, double* y, hipStream_t st) {
  if (P.N2 == 0) return;
  hipLaunchKernelGGL(k_plg_b2, dim3(blocks(P.N2, 256)), dim3(256), 0, st, P, s, e, y);
}
void launch_gather(int n, const int* var_cell, const double* src, double* y, hipStream_t st) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_gather, dim3(blocks(n, 256)), dim3(256), 0, st, n, var_cell, src, y);
}
void launch_lu_forward(const LuDev& F, const LuTasks& T, hipStream_t st) {
  if (T.nF > 0)
    hipLaunchKernelGGL(k_lu_forward, dim3(blocks((long long)T.nF * kWave, 256)), dim3(256), 0, st, F, T.ftask, T.nF);
}
void launch_lu_backward(const LuDev& F, const LuTasks& T, double* out, hipStream_t st) {
  if (T.nB == 0) return;
  hipLaunchKernelGGL(k_lu_backward, dim3(blocks((long long)T.nB * kWave, 256)), dim3(256), 0, st, F, T.btask, T.nB,
                     out);
}
void launch_zero(double* p, long long count, hipStream_t st) {
  if (count == 0) return;
  int nb = (int)std::min<long long>(blocks(count, 256), 8192);
  hipLaunchKernelGGL(k_zero, dim3(nb), dim3(256), 0, st, p, count);
}
void launch_zero_u64(unsigned long long* p, hipStream_t st) {
  hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(1), 0, st, p);
}
void launch_maxabs(const double* v, long long count, unsigned long long* out, hipStream_t st) {
  int nb = (int)std::min<long long>(blocks(count, 256), 2048);
  hipLaunchKernelGGL(k_maxabs, dim3(nb), dim3(256), 0, st, v, count, out);
}
void launch_add_unknowns(const StencilLevel& L, const double* e, double* phi, hipStream_t st) {
  long long n3 = (long long)L.n * L.n * L.n;
  hipLaunchKernelGGL(k_add_unknowns, dim3(blocks(n3, 256)), dim3(256), 0, st, L, e, phi);
}
void launch_mask_unknowns(const StencilLevel& L, double* a, hipStream_t st) {
  long long n3 = (long long)L.n * L.n * L.n;
  hipLaunchKernelGGL(k_mask_unknowns, dim3(blocks(n3, 256)), dim3(256), 0, st, L, a);
}
void launch_copy_pairs(int count, const int2* pairs, double* a, hipStream_t st) {
  if (count == 0) return;
  hipLaunchKernelGGL(k_copy_pairs, dim3(blocks(count, 256)), dim3(256), 0, st, count, pairs, a);
}
void launch_set_values(int count, const int* cells, const double* vals, double* a, hipStream_t st) {
  if (count == 0) return;
  hipLaunchKernelGGL(k_set_values, dim3(blocks(count, 256)), dim3(256), 0, st, count, cells, vals, a);
}
void launch_cell_average(int n, double h, const double* origin, const FieldDesc& f, int mode, int q, double* out,
                         hipStream_t st) {
  GaussQ G;
  G.q = q;
  std::vector<double> x, w;
  gauss_legendre(q, x, w);
  for (int i = 0; i < q; ++i) {
    G.x[i] = x[i];
    G.w[i] = w[i];
  }
  hipLaunchKernelGGL(k_cell_average, grid3(n), kBlock3, 0, st, n, h, origin[0], origin[1], origin[2], f, mode, G,
                     out);
}

}  // namespace cc
