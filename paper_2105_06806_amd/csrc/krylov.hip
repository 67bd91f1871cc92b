// Krylov-vector kernels of the Lanczos recurrence (Sec. 6 "Diagonalization"):
// start vector, FP64-accumulated dot products with a deterministic two-stage
// reduction (per-block partials, then one block in fixed order), the fused
// three-term update w <- w - alpha v_j - beta v_{j-1} with |w|^2, and the
// Gram-Schmidt kernels of the precision mode.
//
// Lanczos vectors are kept unnormalised: vector j is u_j with a device scale
// s_j = 1 / |u_j|, so v_j = s_j u_j and no separate normalisation pass is needed.
// Every kernel reads its scalars (alpha, beta, scales, coefficients) from device
// memory, so a whole Lanczos step is enqueued without a host round trip.
#include <algorithm>
#include <cmath>

#include "common.h"
#include "edx_internal.h"

namespace edx {

namespace {

constexpr int kThreads = 256;
constexpr int kMaxElemBlocks = 1024;

// element (r, c) of a vector with column stride ld draws counter r + c*dup, so
// the start vector is the same for every ld; padding rows are zero
// src (nullable): a dense caller vector copied into the padded layout instead
template <typename T>
__global__ __launch_bounds__(kThreads) void k_start(T* __restrict__ u, int64_t dup, int64_t ld,
                                                    int64_t n, uint64_t seed,
                                                    double* __restrict__ partial,
                                                    const T* __restrict__ src) {
  __shared__ double red[kThreads / 64];
  double acc = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kThreads) {
    const int64_t c = i / ld, r = i - c * ld;
    T t = T(0);
    if (r < dup) {
      if (src) {
        t = src[r + c * dup];
      } else {
        const uint64_t z = splitmix64(seed, (uint64_t)(r + c * dup));
        const double x = (double)(z >> 11) * 0x1.0p-53 * 2.0 - 1.0;
        t = (T)x;
      }
    }
    u[i] = t;
    acc += (double)t * (double)t;
  }
  const double s = block_sum(acc, red);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

__global__ __launch_bounds__(kThreads) void k_reduce_kernel(const double* __restrict__ partial,
                                                            int nparts, int stride,
                                                            double* __restrict__ out, int mode,
                                                            double* __restrict__ out2) {
  __shared__ double red[kThreads / 64];
  const int slot = blockIdx.x;
  double acc = 0.0;
  for (int i = threadIdx.x; i < nparts; i += kThreads) acc += partial[(int64_t)slot * stride + i];
  const double s = block_sum(acc, red);
  if (threadIdx.x == 0) {
    if (mode == 2) {            // beta: sqrt of |w|^2 and the next scale
      const double b = sqrt(s > 0.0 ? s : 0.0);
      out[slot] = b;
      out2[slot] = b > 0.0 ? 1.0 / b : 0.0;
    } else {
      out[slot] = s;
    }
  }
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_update_kernel(
    T* __restrict__ w, const T* __restrict__ vc, const double* __restrict__ scur,
    const T* __restrict__ vp, const double* __restrict__ sprev,
    const double* __restrict__ alpha, const double* __restrict__ beta, int64_t n,
    T* __restrict__ psi, const double* __restrict__ ycoef, double* __restrict__ partial) {
  __shared__ double red[kThreads / 64];
  const double ac = (*alpha) * (*scur);
  const double bp = vp ? (*beta) * (*sprev) : 0.0;
  const double yc = psi ? (*ycoef) * (*scur) : 0.0;
  double acc = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kThreads) {
    const double x = (double)vc[i];
    double r = (double)w[i] - ac * x;
    if (vp) r -= bp * (double)vp[i];
    const T t = (T)r;
    w[i] = t;
    acc += (double)t * (double)t;
    if (psi) psi[i] = (T)((double)psi[i] + yc * x);
  }
  const double s = block_sum(acc, red);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// The same update on 16-byte vectors (4 FP32 or 2 FP64 elements a lane):
// with at most kMaxElemBlocks blocks a CU holds 16 waves, and 4-byte FP32
// lanes left too few bytes in flight to stream at the copy rate (Ns=15 7/7,
// D = 41.4M: 170 us for 666 MB, against 228 us for the 1.33 GB of FP64).
// Requires every vector 16-byte aligned; elements past the last full vector
// are done by scalar lanes.  Each lane sums its elements' squares in element
// order, so the result is deterministic for a given n and grid.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_update_vec_kernel(
    T* __restrict__ w, const T* __restrict__ vc, const double* __restrict__ scur,
    const T* __restrict__ vp, const double* __restrict__ sprev,
    const double* __restrict__ alpha, const double* __restrict__ beta, int64_t n,
    T* __restrict__ psi, const double* __restrict__ ycoef, double* __restrict__ partial) {
  constexpr int V = 16 / (int)sizeof(T);
  typedef T VT __attribute__((ext_vector_type(V)));
  __shared__ double red[kThreads / 64];
  const double ac = (*alpha) * (*scur);
  const double bp = vp ? (*beta) * (*sprev) : 0.0;
  const double yc = psi ? (*ycoef) * (*scur) : 0.0;
  VT* __restrict__ wv = reinterpret_cast<VT*>(w);
  const VT* __restrict__ cv = reinterpret_cast<const VT*>(vc);
  const VT* __restrict__ pv = reinterpret_cast<const VT*>(vp);
  VT* __restrict__ sv = reinterpret_cast<VT*>(psi);
  const int64_t nv = n / V;
  const int64_t stride = (int64_t)gridDim.x * kThreads;
  double acc = 0.0;
  for (int64_t q = blockIdx.x * (int64_t)kThreads + threadIdx.x; q < nv; q += stride) {
    const VT x = cv[q];
    const VT a = wv[q];
    VT b = {};
    if (vp) b = pv[q];
    VT out;
#pragma unroll
    for (int k = 0; k < V; ++k) {
      double r = (double)a[k] - ac * (double)x[k];
      if (vp) r -= bp * (double)b[k];
      const T t = (T)r;
      out[k] = t;
      acc += (double)t * (double)t;
    }
    wv[q] = out;
    if (psi) {
      VT y = sv[q];
#pragma unroll
      for (int k = 0; k < V; ++k) y[k] = (T)((double)y[k] + yc * (double)x[k]);
      sv[q] = y;
    }
  }
  for (int64_t i = nv * V + blockIdx.x * (int64_t)kThreads + threadIdx.x; i < n; i += stride) {
    const double x = (double)vc[i];
    double r = (double)w[i] - ac * x;
    if (vp) r -= bp * (double)vp[i];
    const T t = (T)r;
    w[i] = t;
    acc += (double)t * (double)t;
    if (psi) psi[i] = (T)((double)psi[i] + yc * x);
  }
  const double s = block_sum(acc, red);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_norm2_kernel(const T* __restrict__ x, int64_t n,
                                                           double* __restrict__ partial) {
  __shared__ double red[kThreads / 64];
  double acc = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kThreads) {
    const double t = (double)x[i];
    acc += t * t;
  }
  const double s = block_sum(acc, red);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_scale_copy_kernel(const T* __restrict__ x,
                                                                const double* __restrict__ sc,
                                                                T* __restrict__ y, int64_t n) {
  const double s = *sc;
  for (int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kThreads)
    y[i] = (T)((double)x[i] * s);
}

// partial[0][b] = <w, sa a>, partial[1][b] = <w, sb b>
template <typename T>
__global__ __launch_bounds__(kThreads) void k_dot2_kernel(const T* __restrict__ w,
                                                          const T* __restrict__ a,
                                                          const double* __restrict__ sa,
                                                          const T* __restrict__ b,
                                                          const double* __restrict__ sb,
                                                          int64_t n, double* __restrict__ partial,
                                                          int stride) {
  __shared__ double red[kThreads / 64];
  double da = 0.0, db = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kThreads) {
    const double x = (double)w[i];
    da += x * (double)a[i];
    if (b) db += x * (double)b[i];
  }
  const double s1 = block_sum(da, red);
  const double s2 = block_sum(db, red);
  if (threadIdx.x == 0) {
    partial[blockIdx.x] = s1 * (*sa);
    partial[stride + blockIdx.x] = b ? s2 * (*sb) : 0.0;
  }
}

// w -= ca sa a + cb sb b; partial |w|^2
template <typename T>
__global__ __launch_bounds__(kThreads) void k_axpy2_kernel(
    T* __restrict__ w, const T* __restrict__ a, const double* __restrict__ ca,
    const double* __restrict__ sa, const T* __restrict__ b, const double* __restrict__ cb,
    const double* __restrict__ sb, int64_t n, double* __restrict__ partial) {
  __shared__ double red[kThreads / 64];
  const double fa = (*ca) * (*sa);
  const double fb = b ? (*cb) * (*sb) : 0.0;
  double acc = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kThreads) {
    double r = (double)w[i] - fa * (double)a[i];
    if (b) r -= fb * (double)b[i];
    const T t = (T)r;
    w[i] = t;
    acc += (double)t * (double)t;
  }
  const double s = block_sum(acc, red);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// Full re-orthogonalisation: partial[k][b] = <basis_k, w> for k < m.  Row y
// of the grid takes basis vectors 8y .. 8y + 7 (one pass over w each), so
// small sectors with long bases still spread over the chip; block (x, y)
// sums the same elements in the same order for every y.
constexpr int kMultiChunk = 8;   // basis vectors per pass over w
template <typename T>
__global__ __launch_bounds__(kThreads) void k_multi_dot_kernel(const T* __restrict__ basis,
                                                               int64_t ld, int m,
                                                               const T* __restrict__ w,
                                                               int64_t n,
                                                               double* __restrict__ partial,
                                                               int stride) {
  __shared__ double red[kThreads / 64];
  {
    const int k0 = blockIdx.y * kMultiChunk;   // this row of the grid: basis k0 .. k0 + 7
    double acc[kMultiChunk];
#pragma unroll
    for (int c = 0; c < kMultiChunk; ++c) acc[c] = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kThreads) {
      const double x = (double)w[i];
#pragma unroll
      for (int c = 0; c < kMultiChunk; ++c)
        if (k0 + c < m) acc[c] += x * (double)basis[(int64_t)(k0 + c) * ld + i];
    }
    for (int c = 0; c < kMultiChunk && k0 + c < m; ++c) {
      const double s = block_sum(acc[c], red);
      if (threadIdx.x == 0) partial[(int64_t)(k0 + c) * stride + blockIdx.x] = s;
    }
  }
}

// w -= sum_k coef[k] basis_k; partial |w|^2
template <typename T>
__global__ __launch_bounds__(kThreads) void k_multi_axpy_kernel(T* __restrict__ w,
                                                                const T* __restrict__ basis,
                                                                int64_t ld, int m,
                                                                const double* __restrict__ coef,
                                                                int64_t n,
                                                                double* __restrict__ partial) {
  __shared__ double red[kThreads / 64];
  double acc = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kThreads) {
    double r = (double)w[i];
    for (int k = 0; k < m; ++k) r -= coef[k] * (double)basis[(int64_t)k * ld + i];
    const T t = (T)r;
    w[i] = t;
    acc += (double)t * (double)t;
  }
  const double s = block_sum(acc, red);
  if (partial && threadIdx.x == 0) partial[blockIdx.x] = s;
}

// 16-byte-lane versions of the four Gram-Schmidt kernels above (the same
// reason and requirement as k_update_vec_kernel: every vector 16-byte
// aligned, and so the basis stride; the elements past the last full vector
// are done by scalar lanes).
template <typename T>
using Vec16 = T __attribute__((ext_vector_type(16 / sizeof(T))));

template <typename T>
__global__ __launch_bounds__(kThreads) void k_dot2_vec_kernel(const T* __restrict__ w,
                                                              const T* __restrict__ a,
                                                              const double* __restrict__ sa,
                                                              const T* __restrict__ b,
                                                              const double* __restrict__ sb,
                                                              int64_t n, double* __restrict__ partial,
                                                              int stride) {
  constexpr int V = 16 / (int)sizeof(T);
  __shared__ double red[kThreads / 64];
  const Vec16<T>* __restrict__ wv = reinterpret_cast<const Vec16<T>*>(w);
  const Vec16<T>* __restrict__ av = reinterpret_cast<const Vec16<T>*>(a);
  const Vec16<T>* __restrict__ bv = reinterpret_cast<const Vec16<T>*>(b);
  const int64_t nv = n / V, step = (int64_t)gridDim.x * kThreads;
  double da = 0.0, db = 0.0;
  for (int64_t q = blockIdx.x * (int64_t)kThreads + threadIdx.x; q < nv; q += step) {
    const Vec16<T> x = wv[q], y = av[q];
    Vec16<T> z = {};
    if (b) z = bv[q];
#pragma unroll
    for (int k = 0; k < V; ++k) {
      da += (double)x[k] * (double)y[k];
      if (b) db += (double)x[k] * (double)z[k];
    }
  }
  for (int64_t i = nv * V + blockIdx.x * (int64_t)kThreads + threadIdx.x; i < n; i += step) {
    const double x = (double)w[i];
    da += x * (double)a[i];
    if (b) db += x * (double)b[i];
  }
  const double s1 = block_sum(da, red);
  const double s2 = block_sum(db, red);
  if (threadIdx.x == 0) {
    partial[blockIdx.x] = s1 * (*sa);
    partial[stride + blockIdx.x] = b ? s2 * (*sb) : 0.0;
  }
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_axpy2_vec_kernel(
    T* __restrict__ w, const T* __restrict__ a, const double* __restrict__ ca,
    const double* __restrict__ sa, const T* __restrict__ b, const double* __restrict__ cb,
    const double* __restrict__ sb, int64_t n, double* __restrict__ partial) {
  constexpr int V = 16 / (int)sizeof(T);
  __shared__ double red[kThreads / 64];
  const double fa = (*ca) * (*sa);
  const double fb = b ? (*cb) * (*sb) : 0.0;
  Vec16<T>* __restrict__ wv = reinterpret_cast<Vec16<T>*>(w);
  const Vec16<T>* __restrict__ av = reinterpret_cast<const Vec16<T>*>(a);
  const Vec16<T>* __restrict__ bv = reinterpret_cast<const Vec16<T>*>(b);
  const int64_t nv = n / V, step = (int64_t)gridDim.x * kThreads;
  double acc = 0.0;
  for (int64_t q = blockIdx.x * (int64_t)kThreads + threadIdx.x; q < nv; q += step) {
    const Vec16<T> x = wv[q], y = av[q];
    Vec16<T> z = {};
    if (b) z = bv[q];
    Vec16<T> out;
#pragma unroll
    for (int k = 0; k < V; ++k) {
      double r = (double)x[k] - fa * (double)y[k];
      if (b) r -= fb * (double)z[k];
      out[k] = (T)r;
      acc += (double)out[k] * (double)out[k];
    }
    wv[q] = out;
  }
  for (int64_t i = nv * V + blockIdx.x * (int64_t)kThreads + threadIdx.x; i < n; i += step) {
    double r = (double)w[i] - fa * (double)a[i];
    if (b) r -= fb * (double)b[i];
    const T t = (T)r;
    w[i] = t;
    acc += (double)t * (double)t;
  }
  const double s = block_sum(acc, red);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_multi_dot_vec_kernel(const T* __restrict__ basis,
                                                                   int64_t ld, int m,
                                                                   const T* __restrict__ w,
                                                                   int64_t n,
                                                                   double* __restrict__ partial,
                                                                   int stride) {
  constexpr int V = 16 / (int)sizeof(T);
  __shared__ double red[kThreads / 64];
  const Vec16<T>* __restrict__ wv = reinterpret_cast<const Vec16<T>*>(w);
  const Vec16<T>* __restrict__ bv = reinterpret_cast<const Vec16<T>*>(basis);
  const int64_t nv = n / V, ldv = ld / V, step = (int64_t)gridDim.x * kThreads;
  {
    const int k0 = blockIdx.y * kMultiChunk;   // this row of the grid: basis k0 .. k0 + 7
    double acc[kMultiChunk];
#pragma unroll
    for (int c = 0; c < kMultiChunk; ++c) acc[c] = 0.0;
    for (int64_t q = blockIdx.x * (int64_t)kThreads + threadIdx.x; q < nv; q += step) {
      const Vec16<T> x = wv[q];
#pragma unroll
      for (int c = 0; c < kMultiChunk; ++c)
        if (k0 + c < m) {
          const Vec16<T> y = bv[(int64_t)(k0 + c) * ldv + q];
#pragma unroll
          for (int k = 0; k < V; ++k) acc[c] += (double)x[k] * (double)y[k];
        }
    }
    for (int64_t i = nv * V + blockIdx.x * (int64_t)kThreads + threadIdx.x; i < n; i += step) {
      const double x = (double)w[i];
#pragma unroll
      for (int c = 0; c < kMultiChunk; ++c)
        if (k0 + c < m) acc[c] += x * (double)basis[(int64_t)(k0 + c) * ld + i];
    }
    for (int c = 0; c < kMultiChunk && k0 + c < m; ++c) {
      const double s = block_sum(acc[c], red);
      if (threadIdx.x == 0) partial[(int64_t)(k0 + c) * stride + blockIdx.x] = s;
    }
  }
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_multi_axpy_vec_kernel(T* __restrict__ w,
                                                                    const T* __restrict__ basis,
                                                                    int64_t ld, int m,
                                                                    const double* __restrict__ coef,
                                                                    int64_t n,
                                                                    double* __restrict__ partial) {
  constexpr int V = 16 / (int)sizeof(T);
  __shared__ double red[kThreads / 64];
  Vec16<T>* __restrict__ wv = reinterpret_cast<Vec16<T>*>(w);
  const Vec16<T>* __restrict__ bv = reinterpret_cast<const Vec16<T>*>(basis);
  const int64_t nv = n / V, ldv = ld / V, step = (int64_t)gridDim.x * kThreads;
  double acc = 0.0;
  for (int64_t q = blockIdx.x * (int64_t)kThreads + threadIdx.x; q < nv; q += step) {
    const Vec16<T> x = wv[q];
    double r[V];
#pragma unroll
    for (int k = 0; k < V; ++k) r[k] = (double)x[k];
#pragma unroll 8
    for (int j = 0; j < m; ++j) {
      const Vec16<T> y = bv[(int64_t)j * ldv + q];
      const double c = coef[j];
#pragma unroll
      for (int k = 0; k < V; ++k) r[k] -= c * (double)y[k];
    }
    Vec16<T> out;
#pragma unroll
    for (int k = 0; k < V; ++k) {
      out[k] = (T)r[k];
      acc += (double)out[k] * (double)out[k];
    }
    wv[q] = out;
  }
  for (int64_t i = nv * V + blockIdx.x * (int64_t)kThreads + threadIdx.x; i < n; i += step) {
    double r = (double)w[i];
    for (int j = 0; j < m; ++j) r -= coef[j] * (double)basis[(int64_t)j * ld + i];
    const T t = (T)r;
    w[i] = t;
    acc += (double)t * (double)t;
  }
  const double s = block_sum(acc, red);
  if (partial && threadIdx.x == 0) partial[blockIdx.x] = s;
}

// In-place change of basis for a thick restart: basis_c <- sum_{j<m} C[j][c] basis_j
// for c < l (C row-major, m x l, l <= kMaxKeep).  Each thread owns its
// elements and reads all m of them before it writes, so the overwrite is safe.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_basis_rotate_kernel(T* __restrict__ basis,
                                                                  int64_t ld, int m, int l,
                                                                  const double* __restrict__ C,
                                                                  int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kThreads) {
    double acc[kMaxKeep];
#pragma unroll
    for (int c = 0; c < kMaxKeep; ++c) acc[c] = 0.0;
    for (int j = 0; j < m; ++j) {
      const double x = (double)basis[(int64_t)j * ld + i];
#pragma unroll
      for (int c = 0; c < kMaxKeep; ++c)
        if (c < l) acc[c] += C[(int64_t)j * l + c] * x;
    }
#pragma unroll
    for (int c = 0; c < kMaxKeep; ++c)
      if (c < l) basis[(int64_t)c * ld + i] = (T)acc[c];
  }
}

// coef[k] *= scale[k]^2: <v_k, w> v_k = s_k^2 <u_k, w> u_k for unnormalised u_k
__global__ void k_coef_scale2_kernel(double* __restrict__ coef, const double* __restrict__ scale,
                                     int m) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < m) coef[k] *= scale[k] * scale[k];
}

}  // namespace

edx_status k_coef_scale2(double* coef, const double* scale, int m, hipStream_t st) {
  hipLaunchKernelGGL(k_coef_scale2_kernel, dim3((m + 255) / 256), dim3(256), 0, st, coef, scale,
                     m);
  EDX_HIP(hipGetLastError());
  return EDX_OK;
}

int elem_blocks(int64_t n) {
  int64_t b = (n + kThreads * 4 - 1) / (kThreads * 4);
  return (int)std::max<int64_t>(1, std::min<int64_t>(b, kMaxElemBlocks));
}

// blocks of the full re-orthogonalisation kernels: one element a thread for
// small sectors (their bases are long and the grid would otherwise hold a few
// blocks), the element-kernel cap for large ones
int multi_blocks(int64_t n) {
  const int64_t b = (n + kThreads - 1) / kThreads;
  return (int)std::max<int64_t>(1, std::min<int64_t>(b, kMaxElemBlocks));
}

// every non-null pointer 16-byte aligned (the vector-lane kernels)
template <typename... P>
bool aligned16(const P*... p) {
  return ((reinterpret_cast<uintptr_t>(p) | ... | uintptr_t(0)) & 15) == 0;
}

#define EDX_DISPATCH(vtype, KERN, GRID, ...)                                           \
  do {                                                                                 \
    if ((vtype) == EDX_F64)                                                            \
      hipLaunchKernelGGL(KERN<double>, dim3(GRID), dim3(kThreads), 0, st, __VA_ARGS__); \
    else                                                                               \
      hipLaunchKernelGGL(KERN<float>, dim3(GRID), dim3(kThreads), 0, st, __VA_ARGS__);  \
    EDX_HIP(hipGetLastError());                                                        \
  } while (0)

#define PT(x) reinterpret_cast<T*>(x)

edx_status k_start_vector(int vtype, void* u, int64_t dup, int64_t ld, int64_t ddw,
                          uint64_t seed, double* partial, hipStream_t st, const void* src) {
  const int64_t n = ld * ddw;
  const int g = elem_blocks(n);
  if (vtype == EDX_F64)
    hipLaunchKernelGGL(k_start<double>, dim3(g), dim3(kThreads), 0, st, (double*)u, dup, ld, n,
                       seed, partial, (const double*)src);
  else
    hipLaunchKernelGGL(k_start<float>, dim3(g), dim3(kThreads), 0, st, (float*)u, dup, ld, n,
                       seed, partial, (const float*)src);
  EDX_HIP(hipGetLastError());
  return EDX_OK;
}

namespace {
template <typename T>
__global__ __launch_bounds__(kThreads) void k_unpad_kernel(const T* __restrict__ x, int64_t ld,
                                                           int64_t dup, int64_t n,
                                                           const double* __restrict__ scale,
                                                           T* __restrict__ y) {
  const T sc = (T)(*scale);
  for (int64_t j = blockIdx.x * (int64_t)kThreads + threadIdx.x; j < n;
       j += (int64_t)gridDim.x * kThreads) {
    const int64_t c = j / dup, r = j - c * dup;
    y[j] = x[r + c * ld] * sc;
  }
}
}  // namespace

edx_status k_unpad_scale(int vtype, const void* x, int64_t ld, int64_t dup, int64_t ddw,
                         const double* scale, void* y, hipStream_t st) {
  const int64_t n = dup * ddw;
  const int g = (int)std::max<int64_t>(1, std::min<int64_t>((n + kThreads - 1) / kThreads, 8192));
  if (vtype == EDX_F64)
    hipLaunchKernelGGL(k_unpad_kernel<double>, dim3(g), dim3(kThreads), 0, st, (const double*)x,
                       ld, dup, n, scale, (double*)y);
  else
    hipLaunchKernelGGL(k_unpad_kernel<float>, dim3(g), dim3(kThreads), 0, st, (const float*)x, ld,
                       dup, n, scale, (float*)y);
  EDX_HIP(hipGetLastError());
  return EDX_OK;
}

edx_status k_reduce(const double* partial, int nparts, int nslots, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_reduce_kernel, dim3(nslots), dim3(kThreads), 0, st, partial, nparts,
                     kMaxPartials, out, 0, (double*)nullptr);
  EDX_HIP(hipGetLastError());
  return EDX_OK;
}

edx_status k_reduce_strided(const double* partial, int nparts, int stride, int nslots,
                            double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_reduce_kernel, dim3(nslots), dim3(kThreads), 0, st, partial, nparts,
                     stride, out, 0, (double*)nullptr);
  EDX_HIP(hipGetLastError());
  return EDX_OK;
}

edx_status k_alpha_finish(const double* partial, int nparts, double* alpha_j, hipStream_t st) {
  hipLaunchKernelGGL(k_reduce_kernel, dim3(1), dim3(kThreads), 0, st, partial, nparts, 0,
                     alpha_j, 0, (double*)nullptr);
  EDX_HIP(hipGetLastError());
  return EDX_OK;
}

edx_status k_beta_finish(const double* partial, int nparts, double* beta_next,
                         double* scale_next, hipStream_t st) {
  hipLaunchKernelGGL(k_reduce_kernel, dim3(1), dim3(kThreads), 0, st, partial, nparts, 0,
                     beta_next, 2, scale_next);
  EDX_HIP(hipGetLastError());
  return EDX_OK;
}

edx_status k_update(int vtype, void* w, const void* vcur, const double* scur, const void* vprev,
                    const double* sprev, const double* alpha, const double* beta, int64_t n,
                    void* psi, const double* ycoef, double* partial, hipStream_t st) {
  const int g = elem_blocks(n);
  // 16-byte vector lanes when every vector allows them (workspace vectors are
  // 256-byte aligned), else the element-wise kernel
  const bool vec = aligned16(w, vcur, vprev, psi);
  if (vtype == EDX_F64) {
    auto kern = vec ? k_update_vec_kernel<double> : k_update_kernel<double>;
    hipLaunchKernelGGL(kern, dim3(g), dim3(kThreads), 0, st, (double*)w, (const double*)vcur, scur,
                       (const double*)vprev, sprev, alpha, beta, n, (double*)psi, ycoef, partial);
  } else {
    auto kern = vec ? k_update_vec_kernel<float> : k_update_kernel<float>;
    hipLaunchKernelGGL(kern, dim3(g), dim3(kThreads), 0, st, (float*)w, (const float*)vcur, scur,
                       (const float*)vprev, sprev, alpha, beta, n, (float*)psi, ycoef, partial);
  }
  EDX_HIP(hipGetLastError());
  return EDX_OK;
}

edx_status k_norm2(int vtype, const void* x, int64_t n, double* partial, hipStream_t st) {
  const int g = elem_blocks(n);
  if (vtype == EDX_F64)
    hipLaunchKernelGGL(k_norm2_kernel<double>, dim3(g), dim3(kThreads), 0, st,
                       (const double*)x, n, partial);
  else
    hipLaunchKernelGGL(k_norm2_kernel<float>, dim3(g), dim3(kThreads), 0, st, (const float*)x,
                       n, partial);
  EDX_HIP(hipGetLastError());
  return EDX_OK;
}

edx_status k_scale_copy(int vtype, const void* x, const double* scale, void* y, int64_t n,
                        hipStream_t st) {
  const int g = elem_blocks(n);
  if (vtype == EDX_F64)
    hipLaunchKernelGGL(k_scale_copy_kernel<double>, dim3(g), dim3(kThreads), 0, st,
                       (const double*)x, scale, (double*)y, n);
  else
    hipLaunchKernelGGL(k_scale_copy_kernel<float>, dim3(g), dim3(kThreads), 0, st,
                       (const float*)x, scale, (float*)y, n);
  EDX_HIP(hipGetLastError());
  return EDX_OK;
}

edx_status k_dot2(int vtype, const void* w, const void* a, const double* sa, const void* b,
                  const double* sb, int64_t n, double* partial, hipStream_t st) {
  const int g = elem_blocks(n);
  const bool vec = aligned16(w, a, b);
  if (vtype == EDX_F64) {
    auto kern = vec ? k_dot2_vec_kernel<double> : k_dot2_kernel<double>;
    hipLaunchKernelGGL(kern, dim3(g), dim3(kThreads), 0, st, (const double*)w, (const double*)a,
                       sa, (const double*)b, sb, n, partial, kMaxPartials);
  } else {
    auto kern = vec ? k_dot2_vec_kernel<float> : k_dot2_kernel<float>;
    hipLaunchKernelGGL(kern, dim3(g), dim3(kThreads), 0, st, (const float*)w, (const float*)a,
                       sa, (const float*)b, sb, n, partial, kMaxPartials);
  }
  EDX_HIP(hipGetLastError());
  return EDX_OK;
}

edx_status k_axpy2(int vtype, void* w, const void* a, const double* ca, const double* sa,
                   const void* b, const double* cb, const double* sb, int64_t n,
                   double* partial, hipStream_t st) {
  const int g = elem_blocks(n);
  const bool vec = aligned16(w, a, b);
  if (vtype == EDX_F64) {
    auto kern = vec ? k_axpy2_vec_kernel<double> : k_axpy2_kernel<double>;
    hipLaunchKernelGGL(kern, dim3(g), dim3(kThreads), 0, st, (double*)w, (const double*)a, ca, sa,
                       (const double*)b, cb, sb, n, partial);
  } else {
    auto kern = vec ? k_axpy2_vec_kernel<float> : k_axpy2_kernel<float>;
    hipLaunchKernelGGL(kern, dim3(g), dim3(kThreads), 0, st, (float*)w, (const float*)a, ca, sa,
                       (const float*)b, cb, sb, n, partial);
  }
  EDX_HIP(hipGetLastError());
  return EDX_OK;
}

edx_status k_multi_dot(int vtype, const void* basis, int64_t ld, int m, const void* w, int64_t n,
                       double* partial, hipStream_t st) {
  const int g = multi_blocks(n);
  const bool vec = aligned16(basis, w) && (ld * vbytes(vtype)) % 16 == 0;
  if (m < 1) return EDX_OK;
  const dim3 grid((unsigned)g, (unsigned)((m + kMultiChunk - 1) / kMultiChunk));
  if (vtype == EDX_F64) {
    auto kern = vec ? k_multi_dot_vec_kernel<double> : k_multi_dot_kernel<double>;
    hipLaunchKernelGGL(kern, grid, dim3(kThreads), 0, st, (const double*)basis, ld, m,
                       (const double*)w, n, partial, kMaxPartials);
  } else {
    auto kern = vec ? k_multi_dot_vec_kernel<float> : k_multi_dot_kernel<float>;
    hipLaunchKernelGGL(kern, grid, dim3(kThreads), 0, st, (const float*)basis, ld, m,
                       (const float*)w, n, partial, kMaxPartials);
  }
  EDX_HIP(hipGetLastError());
  return EDX_OK;
}

edx_status k_basis_rotate(int vtype, void* basis, int64_t ld, int m, int l, const double* C,
                          int64_t n, hipStream_t st) {
  if (l < 1 || l > kMaxKeep || m < l) {
    set_error("basis_rotate: need 1 <= l <= " + std::to_string(kMaxKeep) + " and l <= m");
    return EDX_E_INVALID;
  }
  const int g = elem_blocks(n);
  if (vtype == EDX_F64)
    hipLaunchKernelGGL(k_basis_rotate_kernel<double>, dim3(g), dim3(kThreads), 0, st,
                       (double*)basis, ld, m, l, C, n);
  else
    hipLaunchKernelGGL(k_basis_rotate_kernel<float>, dim3(g), dim3(kThreads), 0, st,
                       (float*)basis, ld, m, l, C, n);
  EDX_HIP(hipGetLastError());
  return EDX_OK;
}

edx_status k_multi_axpy(int vtype, void* w, const void* basis, int64_t ld, int m,
                        const double* coef, int64_t n, double* partial, hipStream_t st) {
  const int g = multi_blocks(n);
  const bool vec = aligned16(w, basis) && (ld * vbytes(vtype)) % 16 == 0;
  if (vtype == EDX_F64) {
    auto kern = vec ? k_multi_axpy_vec_kernel<double> : k_multi_axpy_kernel<double>;
    hipLaunchKernelGGL(kern, dim3(g), dim3(kThreads), 0, st, (double*)w, (const double*)basis, ld,
                       m, coef, n, partial);
  } else {
    auto kern = vec ? k_multi_axpy_vec_kernel<float> : k_multi_axpy_kernel<float>;
    hipLaunchKernelGGL(kern, dim3(g), dim3(kThreads), 0, st, (float*)w, (const float*)basis, ld,
                       m, coef, n, partial);
  }
  EDX_HIP(hipGetLastError());
  return EDX_OK;
}

}  // namespace edx
