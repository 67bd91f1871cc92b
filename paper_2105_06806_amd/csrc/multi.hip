// Several bath sets of one sector shape at once: the Lanczos ground states of
// K independent impurity problems (the paper's parallelism over independent
// problems, Sec. 6 "Main") whose sectors have the same (Ns, Norb, N_up,
// N_dw) -- so the same strings, hop columns and signs -- but their own bath
// energies, hybridisations and interaction (their own amplitude, energy and
// pattern-pair tables).
//
// Layout: the K vectors are interleaved element by element, element (i, j)
// of set b (row i of column j of eq. Vmatrix, column stride ld) at
// (i + j ld) K + b.  A column of all K sets is then ld K contiguous elements,
// and a spin-down neighbour value of all K sets is K contiguous elements, so
// one gather serves K products (one wide load per lane).
//
// k_hv_multi is the fused pass of the single-vector product with one column
// per workgroup: the column of all K sets is staged in LDS (interleaved, so a
// spin-up hop reads its K values from adjacent words), the spin-down
// neighbours of the column come from global memory K values at a time, and
// each set's result is summed in the same order as the single-vector pass,
// so every set's H v is the single-vector one bit for bit.  The recurrence
// kernels (start vector, three-term update with |w|^2, reductions) work on the
// interleaved vectors with K scalars per step, and the host evaluates the
// stop rule of every set on its own tridiagonal matrix.
#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "common.h"
#include "edx_internal.h"

namespace edx {

bool multi_supported(const edx_sector* s, int K, int vtype);
bool multi_same_shape(const edx_sector* a, const edx_sector* b);

namespace {

constexpr int kMultiThreads = 256;       // recurrence kernels
constexpr int kMultiElemBlocks = 1024;

__host__ __device__ constexpr size_t m_al16(size_t x) { return (x + 15) & ~(size_t)15; }

template <typename T>
struct MultiArgs {
  int64_t dup, ddw, ld;            // ld: column stride of one set, >= dup
  const uint32_t* hdw;             // spin-down hop rows, packed, stride WDW (shared)
  const uint8_t* hrow;             // compact spin-up rows: WUP 16-bit columns, WUP 8-bit
                                   // amplitude indices (shared)
  const uint8_t* pup;              // impurity patterns (shared)
  const uint8_t* pdw;
  const T* amp;                    // [K][256] signed amplitudes of each set
  const T* W;                      // [K][64] pattern-pair interaction of each set
  const T* eup;                    // [K][dup] spin-up string energies of each set
  const T* edw;                    // [K][ddw]
};

// K * sizeof(T) bytes at byte offset voff + soff of the buffer, as b128 /
// b64 / b32 loads
template <typename T, int K>
__device__ __forceinline__ void load_k(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff,
                                       T (&out)[K]) {
  constexpr int B = K * (int)sizeof(T);
  typedef unsigned int u2 __attribute__((ext_vector_type(2)));
  typedef unsigned int u4 __attribute__((ext_vector_type(4)));
  unsigned words[B / 4];
  int o = 0;
#pragma unroll
  for (; o + 16 <= B; o += 16) {
    const u4 x = __builtin_amdgcn_raw_buffer_load_b128(r, (int)(voff + o), (int)soff, 0);
    words[o / 4] = x.x; words[o / 4 + 1] = x.y; words[o / 4 + 2] = x.z; words[o / 4 + 3] = x.w;
  }
#pragma unroll
  for (; o + 8 <= B; o += 8) {
    const u2 x = __builtin_amdgcn_raw_buffer_load_b64(r, (int)(voff + o), (int)soff, 0);
    words[o / 4] = x.x; words[o / 4 + 1] = x.y;
  }
#pragma unroll
  for (; o + 4 <= B; o += 4)
    words[o / 4] = __builtin_amdgcn_raw_buffer_load_b32(r, (int)(voff + o), (int)soff, 0);
#pragma unroll
  for (int b = 0; b < K; ++b) {
    if constexpr (sizeof(T) == 4)
      out[b] = __uint_as_float(words[b]);
    else
      out[b] = __longlong_as_double(
          (long long)(((unsigned long long)words[2 * b + 1] << 32) | words[2 * b]));
  }
}

// streaming store of K values
template <typename T, int K>
__device__ __forceinline__ void store_k(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff,
                                        const T (&x)[K]) {
  constexpr int B = K * (int)sizeof(T);
  typedef unsigned int u2 __attribute__((ext_vector_type(2)));
  typedef unsigned int u4 __attribute__((ext_vector_type(4)));
  unsigned words[B / 4];
#pragma unroll
  for (int b = 0; b < K; ++b) {
    if constexpr (sizeof(T) == 4) {
      words[b] = __float_as_uint(x[b]);
    } else {
      const unsigned long long u = (unsigned long long)__double_as_longlong(x[b]);
      words[2 * b] = (unsigned)u;
      words[2 * b + 1] = (unsigned)(u >> 32);
    }
  }
  int o = 0;
#pragma unroll
  for (; o + 16 <= B; o += 16) {
    u4 y;
    y.x = words[o / 4]; y.y = words[o / 4 + 1]; y.z = words[o / 4 + 2]; y.w = words[o / 4 + 3];
    __builtin_amdgcn_raw_buffer_store_b128(y, r, (int)(voff + o), (int)soff, 2);
  }
#pragma unroll
  for (; o + 8 <= B; o += 8) {
    u2 y;
    y.x = words[o / 4]; y.y = words[o / 4 + 1];
    __builtin_amdgcn_raw_buffer_store_b64(y, r, (int)(voff + o), (int)soff, 2);
  }
#pragma unroll
  for (; o + 4 <= B; o += 4)
    __builtin_amdgcn_raw_buffer_store_b32(words[o / 4], r, (int)(voff + o), (int)soff, 2);
}

__device__ __forceinline__ float m_uniform(float x) {
  return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(x)));
}
__device__ __forceinline__ double m_uniform(double x) {
  const long long b = __double_as_longlong(x);
  const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)b);
  const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(b >> 32));
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// w_b = H_b (vscale_b v_b) for the K sets, column blockIdx.x; partial[b *
// pstride + block] = <vscale_b v_b, w_b> over the column (FP64).  Requires
// ld * ddw * K * sizeof(T) < 2^32 (buffer offsets).
template <typename T, int WUP, int WDW, int K>
__global__ __launch_bounds__(1024) void k_hv_multi(MultiArgs<T> a, const T* __restrict__ v,
                                                   T* __restrict__ w,
                                                   const double* __restrict__ vscale,
                                                   double* __restrict__ partial, int pstride,
                                                   uint32_t vbytes) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int64_t dup = a.dup, ld = a.ld;
  T* vs = reinterpret_cast<T*>(smem_raw);                                   // [dup][K]
  T* amp = reinterpret_cast<T*>(smem_raw + m_al16((size_t)dup * K * sizeof(T)));   // [K][256]
  T* Wt = amp + K * kAmpTable;                                              // [K][64]
  double* red = reinterpret_cast<double*>(Wt + K * 64);                     // [16]
  const int64_t j = blockIdx.x;
  T sc[K];
#pragma unroll
  for (int b = 0; b < K; ++b) sc[b] = vscale ? (T)vscale[b] : T(1);
  __amdgpu_buffer_rsrc_t vres =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<T*>(v), 0, (int)vbytes, 0x00020000);
  __amdgpu_buffer_rsrc_t wres = __builtin_amdgcn_make_buffer_rsrc(w, 0, (int)vbytes, 0x00020000);
  const uint32_t coff =
      __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)j * ld * K * sizeof(T)));
  // stage the column of all K sets (the interleaved LDS image is the global
  // layout of the column), scaled
  for (int64_t r = threadIdx.x; r < dup; r += blockDim.x) {
    T x[K];
    load_k<T, K>(vres, (uint32_t)(r * K * sizeof(T)), coff, x);
#pragma unroll
    for (int b = 0; b < K; ++b) vs[r * K + b] = x[b] * sc[b];
  }
  for (int i = threadIdx.x; i < K * kAmpTable; i += blockDim.x) amp[i] = a.amp[i];
  for (int i = threadIdx.x; i < K * 64; i += blockDim.x) Wt[i] = a.W[i];
  // the column's spin-down neighbours (block-uniform)
  uint32_t goff[WDW];
  T gamp[WDW][K];
#pragma unroll
  for (int k = 0; k < WDW; ++k) {
    const uint32_t f = a.hdw[j * WDW + k];
    goff[k] = __builtin_amdgcn_readfirstlane(
        (uint32_t)((uint64_t)(f & kColMask) * (uint64_t)ld * K * sizeof(T)));
#pragma unroll
    for (int b = 0; b < K; ++b) gamp[k][b] = m_uniform(a.amp[b * kAmpTable + (f >> kAmpShift)] * sc[b]);
  }
  T ed[K];
#pragma unroll
  for (int b = 0; b < K; ++b) ed[b] = a.edw[b * a.ddw + j];
  const int pd = a.pdw[j];
  constexpr int HW = 3 * WUP / 4;   // 32-bit words of a compact spin-up row
  __amdgpu_buffer_rsrc_t hres = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<uint8_t*>(a.hrow), 0, (int)(dup * HW * 4), 0x00020000);
  __syncthreads();
  double dot[K];
#pragma unroll
  for (int b = 0; b < K; ++b) dot[b] = 0.0;
  for (uint32_t iu = threadIdx.x; iu < (uint32_t)dup; iu += blockDim.x) {
    const uint32_t voff = iu * (uint32_t)(K * sizeof(T));
    uint32_t rw[HW];
#pragma unroll
    for (int q = 0; q < HW / 2; ++q) {
      typedef unsigned int u2 __attribute__((ext_vector_type(2)));
      const u2 x = __builtin_amdgcn_raw_buffer_load_b64(hres, (int)(iu * HW * 4 + q * 8), 0, 0);
      rw[2 * q] = x.x;
      rw[2 * q + 1] = x.y;
    }
    T eu[K];
#pragma unroll
    for (int b = 0; b < K; ++b) eu[b] = a.eup[b * dup + iu];
    const int pu = a.pup[iu] * 8;
    uint32_t col[WUP], ai[WUP];
#pragma unroll
    for (int k = 0; k < WUP; ++k) {
      col[k] = (rw[k >> 1] >> (16 * (k & 1))) & 0xFFFFu;
      ai[k] = (rw[WUP / 2 + (k >> 2)] >> (8 * (k & 3))) & 0xFFu;
    }
    T g[WDW][K];
#pragma unroll
    for (int k = 0; k < WDW; ++k) load_k<T, K>(vres, voff, goff[k], g[k]);
    T acc[K];
#pragma unroll
    for (int b = 0; b < K; ++b) acc[b] = T(0);
#pragma unroll
    for (int k = 0; k < WUP; ++k) {
      const T* src = vs + col[k] * K;
#pragma unroll
      for (int b = 0; b < K; ++b) acc[b] += amp[b * kAmpTable + ai[k]] * src[b];
    }
    T res[K];
#pragma unroll
    for (int b = 0; b < K; ++b) {
      const T x = vs[iu * K + b];
      T s2 = T(0);
#pragma unroll
      for (int k = 0; k < WDW; ++k) s2 += gamp[k][b] * g[k][b];
      res[b] = acc[b] + (eu[b] + ed[b] + Wt[b * 64 + pu + pd]) * x + s2;
      dot[b] += (double)x * (double)res[b];
    }
    store_k<T, K>(wres, voff, coff, res);
  }
  // padding rows of the output column are zero
  for (int64_t i = dup * K + threadIdx.x; i < ld * K; i += blockDim.x) w[j * ld * K + i] = T(0);
#pragma unroll
  for (int b = 0; b < K; ++b) {
    const double s = block_sum(dot[b], red);
    if (threadIdx.x == 0) partial[(size_t)b * pstride + blockIdx.x] = s;
  }
}

// the same counter-based start vector as the single-set path (SplitMix64 of
// the logical index, one seed for every set); partial[b][block] = |u_b|^2
template <typename T, int K>
__global__ __launch_bounds__(kMultiThreads) void k_mstart(T* __restrict__ u, int64_t dup,
                                                          int64_t ld, int64_t ncol, uint64_t seed,
                                                          double* __restrict__ partial,
                                                          int pstride) {
  __shared__ double red[kMultiThreads / 64];
  const int64_t n = ld * ncol;
  double acc = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)kMultiThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kMultiThreads) {
    const int64_t c = i / ld, r = i - c * ld;
    T t = T(0);
    if (r < dup) {
      const uint64_t z = splitmix64(seed, (uint64_t)(r + c * dup));
      t = (T)((double)(z >> 11) * 0x1.0p-53 * 2.0 - 1.0);
    }
#pragma unroll
    for (int b = 0; b < K; ++b) u[i * K + b] = t;
    acc += (double)t * (double)t;
  }
  const double s = block_sum(acc, red);
  if (threadIdx.x == 0)
    for (int b = 0; b < K; ++b) partial[(size_t)b * pstride + blockIdx.x] = s;
}

// w_b -= alpha_b s_b v_b + beta_b s'_b v'_b (vp may be null), partial[b][block]
// = |w_b|^2; scalars are [K] arrays.  Each thread handles one set's elements
// (the grid stride is a multiple of K).
template <typename T, int K>
__global__ __launch_bounds__(kMultiThreads) void k_mupdate(
    T* __restrict__ w, const T* __restrict__ vc, const double* __restrict__ scur,
    const T* __restrict__ vp, const double* __restrict__ sprev,
    const double* __restrict__ alpha, const double* __restrict__ beta, int64_t n,
    double* __restrict__ partial, int pstride) {
  const int b = threadIdx.x % K;
  const double ac = alpha[b] * scur[b];
  const double bp = vp ? beta[b] * sprev[b] : 0.0;
  double acc = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)kMultiThreads + threadIdx.x; i < n * K;
       i += (int64_t)gridDim.x * kMultiThreads) {
    double r = (double)w[i] - ac * (double)vc[i];
    if (vp) r -= bp * (double)vp[i];
    const T t = (T)r;
    w[i] = t;
    acc += (double)t * (double)t;
  }
  // per-set block sums: lanes with the same b (K divides 64)
  for (int off = K; off < 64; off <<= 1) acc += __shfl_xor(acc, off, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __shared__ double part[kMultiThreads / 64][K];
  if (lane < K) part[wid][lane] = acc;
  __syncthreads();
  if (threadIdx.x < K) {
    double s = 0.0;
    for (int q = 0; q < kMultiThreads / 64; ++q) s += part[q][threadIdx.x];
    partial[(size_t)threadIdx.x * pstride + blockIdx.x] = s;
  }
}

// out[b] = sum of partial[b][0..nparts); mode 1: out = sqrt, out2 = 1/out
// (0 for a vanishing norm)
__global__ __launch_bounds__(kMultiThreads) void k_mreduce(const double* __restrict__ partial,
                                                           int nparts, int pstride,
                                                           double* __restrict__ out,
                                                           double* __restrict__ out2, int mode) {
  __shared__ double red[kMultiThreads / 64];
  const int b = blockIdx.x;
  double s = 0.0;
  for (int i = threadIdx.x; i < nparts; i += kMultiThreads) s += partial[(size_t)b * pstride + i];
  s = block_sum(s, red);
  if (threadIdx.x == 0) {
    if (mode == 1) {
      const double x = sqrt(s > 0.0 ? s : 0.0);
      out[b] = x;
      out2[b] = x > 0.0 ? 1.0 / x : 0.0;
    } else {
      out[b] = s;
    }
  }
}

int m_elem_blocks(int64_t n) {
  int64_t b = (n + kMultiThreads * 4 - 1) / (kMultiThreads * 4);
  return (int)std::max<int64_t>(1, std::min<int64_t>(b, kMultiElemBlocks));
}

size_t multi_lds(int64_t dup, int K, size_t tsz) {
  return m_al16((size_t)dup * K * tsz) + (size_t)K * (kAmpTable + 64) * tsz + 16 * sizeof(double) + 64;
}

template <typename T, int WUP, int WDW, int K>
edx_status launch_multi_k(const MultiArgs<T>& a, const T* v, T* w, const double* vscale,
                          double* partial, int pstride, uint32_t vbytes, hipStream_t st) {
  const size_t lds = multi_lds(a.dup, K, sizeof(T));
  const int nthr = a.dup >= 2048 ? 512 : 256;
  const void* kern = (const void*)k_hv_multi<T, WUP, WDW, K>;
  EDX_HIP(hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  hipLaunchKernelGGL((k_hv_multi<T, WUP, WDW, K>), dim3((unsigned)a.ddw), dim3(nthr), lds, st, a,
                     v, w, vscale, partial, pstride, vbytes);
  EDX_HIP(hipGetLastError());
  return EDX_OK;
}

template <typename T, int K>
edx_status launch_multi_w(const MultiArgs<T>& a, int wup, int wdw, const T* v, T* w,
                          const double* vscale, double* partial, int pstride, uint32_t vbytes,
                          hipStream_t st) {
  if (wup == 8 && wdw == 8)
    return launch_multi_k<T, 8, 8, K>(a, v, w, vscale, partial, pstride, vbytes, st);
  if (wup == 16 && wdw == 16)
    return launch_multi_k<T, 16, 16, K>(a, v, w, vscale, partial, pstride, vbytes, st);
  set_error("multi: hop rows of 8 or 16 entries only");
  return EDX_E_UNSUPPORTED;
}

template <typename T>
edx_status launch_multi(const MultiArgs<T>& a, int K, int wup, int wdw, const T* v, T* w,
                        const double* vscale, double* partial, int pstride, uint32_t vbytes,
                        hipStream_t st) {
  switch (K) {
    case 1: return launch_multi_w<T, 1>(a, wup, wdw, v, w, vscale, partial, pstride, vbytes, st);
    case 2: return launch_multi_w<T, 2>(a, wup, wdw, v, w, vscale, partial, pstride, vbytes, st);
    case 4: return launch_multi_w<T, 4>(a, wup, wdw, v, w, vscale, partial, pstride, vbytes, st);
    case 8: return launch_multi_w<T, 8>(a, wup, wdw, v, w, vscale, partial, pstride, vbytes, st);
    default:
      set_error("multi: K must be 1, 2, 4 or 8");
      return EDX_E_INVALID;
  }
}

template <typename T, int K>
void launch_mstart(T* u, int64_t dup, int64_t ld, int64_t ncol, uint64_t seed, double* partial,
                   int pstride, hipStream_t st) {
  hipLaunchKernelGGL((k_mstart<T, K>), dim3(m_elem_blocks(ld * ncol)), dim3(kMultiThreads), 0,
                     st, u, dup, ld, ncol, seed, partial, pstride);
}

template <typename T, int K>
void launch_mupdate(T* w, const T* vc, const double* sc, const T* vp, const double* sp,
                    const double* al, const double* be, int64_t n, double* partial, int pstride,
                    hipStream_t st) {
  hipLaunchKernelGGL((k_mupdate<T, K>), dim3(m_elem_blocks(n * K)), dim3(kMultiThreads), 0, st,
                     w, vc, sc, vp, sp, al, be, n, partial, pstride);
}

template <typename T>
edx_status mstart(int K, T* u, int64_t dup, int64_t ld, int64_t ncol, uint64_t seed,
                  double* partial, int pstride, hipStream_t st) {
  switch (K) {
    case 1: launch_mstart<T, 1>(u, dup, ld, ncol, seed, partial, pstride, st); break;
    case 2: launch_mstart<T, 2>(u, dup, ld, ncol, seed, partial, pstride, st); break;
    case 4: launch_mstart<T, 4>(u, dup, ld, ncol, seed, partial, pstride, st); break;
    default: launch_mstart<T, 8>(u, dup, ld, ncol, seed, partial, pstride, st); break;
  }
  EDX_HIP(hipGetLastError());
  return EDX_OK;
}

template <typename T>
edx_status mupdate(int K, T* w, const T* vc, const double* sc, const T* vp, const double* sp,
                   const double* al, const double* be, int64_t n, double* partial, int pstride,
                   hipStream_t st) {
  switch (K) {
    case 1: launch_mupdate<T, 1>(w, vc, sc, vp, sp, al, be, n, partial, pstride, st); break;
    case 2: launch_mupdate<T, 2>(w, vc, sc, vp, sp, al, be, n, partial, pstride, st); break;
    case 4: launch_mupdate<T, 4>(w, vc, sc, vp, sp, al, be, n, partial, pstride, st); break;
    default: launch_mupdate<T, 8>(w, vc, sc, vp, sp, al, be, n, partial, pstride, st); break;
  }
  EDX_HIP(hipGetLastError());
  return EDX_OK;
}

// Workspace of a group: 3 interleaved vectors, the per-set tables, partial
// sums and the scalars.
struct MultiWs {
  char* vec[3];
  char* amp;
  char* W;
  char* eup;
  char* edw;
  double* partial;   // [K][pstride]
  int pstride;
  double* alpha;     // [niter + 1][K]
  double* beta;      // [niter + 2][K]
  double* scale;     // [niter + 2][K]
  size_t total;
};

MultiWs multi_layout(const edx_sector* s, int K, int vtype, int niter, char* base) {
  MultiWs M{};
  const size_t tsz = vbytes(vtype);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += align_up(bytes);
    return base ? base + o : nullptr;
  };
  const size_t vb = (size_t)s->vlen * K * tsz;
  for (int q = 0; q < 3; ++q) M.vec[q] = take(vb);
  M.amp = take((size_t)K * kAmpTable * tsz);
  M.W = take((size_t)K * 64 * tsz);
  M.eup = take((size_t)K * s->dup * tsz);
  M.edw = take((size_t)K * s->ddw * tsz);
  M.pstride = (int)std::max<int64_t>(s->ddw, kMultiElemBlocks);
  M.partial = (double*)take(sizeof(double) * (size_t)K * M.pstride);
  M.alpha = (double*)take(sizeof(double) * (size_t)(niter + 2) * K);
  M.beta = (double*)take(sizeof(double) * (size_t)(niter + 2) * K);
  M.scale = (double*)take(sizeof(double) * (size_t)(niter + 2) * K);
  M.total = off;
  return M;
}

// the per-set tables of a group, set-major, into the workspace
edx_status stage_tables(const edx_sector* const* secs, int K, int vtype, const MultiWs& M,
                        hipStream_t st) {
  const size_t tsz = vbytes(vtype);
  const bool f32 = vtype == EDX_F32;
  for (int b = 0; b < K; ++b) {
    const edx_sector* s = secs[b];
    EDX_HIP(hipMemcpyAsync(M.amp + (size_t)b * kAmpTable * tsz,
                           f32 ? (void*)s->amp32 : (void*)s->amp64, kAmpTable * tsz,
                           hipMemcpyDeviceToDevice, st));
    EDX_HIP(hipMemcpyAsync(M.W + (size_t)b * 64 * tsz, f32 ? (void*)s->w32 : (void*)s->w64,
                           64 * tsz, hipMemcpyDeviceToDevice, st));
    EDX_HIP(hipMemcpyAsync(M.eup + (size_t)b * s->dup * tsz,
                           f32 ? (void*)s->up.e32 : (void*)s->up.e64, s->dup * tsz,
                           hipMemcpyDeviceToDevice, st));
    EDX_HIP(hipMemcpyAsync(M.edw + (size_t)b * s->ddw * tsz,
                           f32 ? (void*)s->dw.e32 : (void*)s->dw.e64, s->ddw * tsz,
                           hipMemcpyDeviceToDevice, st));
  }
  return EDX_OK;
}

edx_status check_group(const edx_sector* const* secs, int K, int vtype) {
  if (K != 1 && K != 2 && K != 4 && K != 8) {
    set_error("multi: the number of sets must be 1, 2, 4 or 8");
    return EDX_E_INVALID;
  }
  for (int b = 0; b < K; ++b)
    if (!secs[b]) {
      set_error("multi: a sector handle is NULL");
      return EDX_E_INVALID;
    }
  for (int b = 1; b < K; ++b)
    if (!multi_same_shape(secs[0], secs[b])) {
      set_error("multi: sectors of different shapes");
      return EDX_E_INVALID;
    }
  if (!multi_supported(secs[0], K, vtype)) {
    set_error("multi: sector shape not supported by the multi-set pass");
    return EDX_E_UNSUPPORTED;
  }
  return EDX_OK;
}

}  // namespace

// shapes the multi-set pass handles: total-N electronic sectors (no H_nd, no
// phonons), compact spin-up rows, hop rows of 8 or 16, the column of K sets in
// LDS and 32-bit buffer offsets
bool multi_supported(const edx_sector* s, int K, int vtype) {
  if (!s || s->nd || s->dph > 1 || s->orb || !s->up.hop || !s->hrow) return false;
  if (!((s->up.wpad == 8 && s->dw.wpad == 8) || (s->up.wpad == 16 && s->dw.wpad == 16))) return false;
  if (multi_lds(s->dup, K, vbytes(vtype)) > 160 * 1024) return false;
  return (uint64_t)s->vlen * K * vbytes(vtype) <= 0xFFFFFFFFull;
}

// the same strings, hops and signs (so one table set serves every job)
bool multi_same_shape(const edx_sector* a, const edx_sector* b) {
  return a->model.ns == b->model.ns && a->model.norb == b->model.norb &&
         a->model.nbath == b->model.nbath && a->nup == b->nup && a->ndw == b->ndw &&
         a->dup == b->dup && a->ddw == b->ddw && a->ld == b->ld && !a->orb && !b->orb;
}

size_t multi_workspace_bytes(const edx_sector* s, int K, int vtype, int niter) {
  return multi_layout(s, K, vtype, niter, nullptr).total + 256;
}

// Ground energies of K sectors of one shape (the plain recurrence of
// edx_lanczos_ground_state for each, psi0 not formed): one interleaved
// product and recurrence per step for all K, the stop rule of each set on
// the host every check_every steps (tol, rtol, FP32 floor, breakdown,
// niter), a set's result frozen at its stop while the others go on.
edx_status multi_ground_states(const edx_sector* const* secs, int K, const edx_lanczos_opts* o,
                               void* ws, size_t ws_bytes, edx_batch_result* res, hipStream_t st) {
  const int vtype = o->vtype;
  const int niter = o->niter;
  const edx_sector* s0 = secs[0];
  EDX_TRY(check_group(secs, K, vtype));
  char* base = reinterpret_cast<char*>(align_up(reinterpret_cast<uintptr_t>(ws)));
  const MultiWs M = multi_layout(s0, K, vtype, niter, base);
  if (M.total + (size_t)(base - (char*)ws) > ws_bytes) {
    set_error("multi: workspace too small (need " + std::to_string(M.total + 256) + " bytes)");
    return EDX_E_NOMEM;
  }
  const size_t tsz = vbytes(vtype);
  EDX_TRY(stage_tables(secs, K, vtype, M, st));
  const int64_t n = s0->vlen;
  const uint32_t vbytes32 = (uint32_t)((uint64_t)n * K * tsz);
  const int eb = m_elem_blocks(n * K);
  auto hv = [&](const void* v, void* w, const double* vscale) -> edx_status {
    if (vtype == EDX_F32) {
      MultiArgs<float> a{s0->dup, s0->ddw, s0->ld, s0->dw.hop, s0->hrow, s0->up.pat, s0->dw.pat,
                         (const float*)M.amp, (const float*)M.W, (const float*)M.eup,
                         (const float*)M.edw};
      return launch_multi<float>(a, K, s0->up.wpad, s0->dw.wpad, (const float*)v, (float*)w,
                                 vscale, M.partial, M.pstride, vbytes32, st);
    }
    MultiArgs<double> a{s0->dup, s0->ddw, s0->ld, s0->dw.hop, s0->hrow, s0->up.pat, s0->dw.pat,
                        (const double*)M.amp, (const double*)M.W, (const double*)M.eup,
                        (const double*)M.edw};
    return launch_multi<double>(a, K, s0->up.wpad, s0->dw.wpad, (const double*)v, (double*)w,
                                vscale, M.partial, M.pstride, vbytes32, st);
  };
  auto update = [&](void* w, const void* vc, const double* sc, const void* vp, const double* sp,
                    const double* al, const double* be) -> edx_status {
    if (vtype == EDX_F32)
      return mupdate<float>(K, (float*)w, (const float*)vc, sc, (const float*)vp, sp, al, be, n,
                            M.partial, M.pstride, st);
    return mupdate<double>(K, (double*)w, (const double*)vc, sc, (const double*)vp, sp, al, be,
                           n, M.partial, M.pstride, st);
  };
  // start vectors and their scales
  if (vtype == EDX_F32)
    EDX_TRY(mstart<float>(K, (float*)M.vec[0], s0->dup, s0->ld, s0->ddw, o->seed, M.partial,
                          M.pstride, st));
  else
    EDX_TRY(mstart<double>(K, (double*)M.vec[0], s0->dup, s0->ld, s0->ddw, o->seed, M.partial,
                           M.pstride, st));
  hipLaunchKernelGGL(k_mreduce, dim3(K), dim3(kMultiThreads), 0, st, M.partial,
                     m_elem_blocks(n), M.pstride, M.beta, M.scale, 1);
  EDX_HIP(hipGetLastError());
  EDX_HIP(hipMemsetAsync(M.beta, 0, sizeof(double) * K, st));   // beta_0 couples nothing

  std::vector<double> ha((size_t)(niter + 2) * K), hb((size_t)(niter + 2) * K);
  std::vector<double> ta(niter + 2), tb(niter + 2);
  std::vector<int> done(K, 0);
  std::vector<double> tnorm(K, 0.0), Eold(K, NAN);
  int left = K;
  int steps = 0;
  const int every = std::max(1, o->check_every);
  while (steps < niter && left > 0) {
    const int upto = std::min(niter, steps + every);
    for (int j = steps; j < upto; ++j) {
      const void* cur = M.vec[j % 3];
      const void* prev = j > 0 ? M.vec[(j + 2) % 3] : nullptr;
      void* w = M.vec[(j + 1) % 3];
      EDX_TRY(hv(cur, w, M.scale + (size_t)j * K));
      hipLaunchKernelGGL(k_mreduce, dim3(K), dim3(kMultiThreads), 0, st, M.partial,
                         (int)s0->ddw, M.pstride, M.alpha + (size_t)j * K, (double*)nullptr, 0);
      EDX_HIP(hipGetLastError());
      EDX_TRY(update(w, cur, M.scale + (size_t)j * K, prev,
                     j > 0 ? M.scale + (size_t)(j - 1) * K : nullptr, M.alpha + (size_t)j * K,
                     M.beta + (size_t)j * K));
      hipLaunchKernelGGL(k_mreduce, dim3(K), dim3(kMultiThreads), 0, st, M.partial, eb,
                         M.pstride, M.beta + (size_t)(j + 1) * K, M.scale + (size_t)(j + 1) * K,
                         1);
      EDX_HIP(hipGetLastError());
    }
    EDX_HIP(hipMemcpyAsync(ha.data(), M.alpha, sizeof(double) * (size_t)upto * K,
                           hipMemcpyDeviceToHost, st));
    EDX_HIP(hipMemcpyAsync(hb.data(), M.beta, sizeof(double) * (size_t)(upto + 1) * K,
                           hipMemcpyDeviceToHost, st));
    EDX_HIP(hipStreamSynchronize(st));
    for (int b = 0; b < K; ++b) {
      if (done[b]) continue;
      for (int q = 0; q <= upto; ++q) {
        if (q < upto) ta[q] = ha[(size_t)q * K + b];
        tb[q] = hb[(size_t)q * K + b];
      }
      for (int j = steps; j < upto && !done[b]; ++j) {
        // the stop rule of the single-set path (FP32 floor included)
        tnorm[b] = std::max(tnorm[b], std::fabs(ta[j]) + tb[j] + tb[j + 1]);
        const double E = tridiag_lowest(ta.data(), tb.data() + 1, j + 1, 0);
        const bool bd = !(tb[j + 1] > 1e-12 * tnorm[b]);
        const double floor32 = vtype == EDX_F32 ? 2.0 * 1.1920929e-7 * tnorm[b] : 0.0;
        bool ok = j > 0 &&
                  std::fabs(E - Eold[b]) <= std::max(o->tol * std::max(1.0, std::fabs(E)), floor32);
        if (ok && o->rtol > 0.0) {
          std::vector<double> yv(j + 1);
          tridiag_vector(ta.data(), tb.data() + 1, j + 1, E, yv.data());
          const double resid = tb[j + 1] * std::fabs(yv[j]);
          ok = resid <= std::max(o->rtol * std::max(1.0, std::fabs(E)), floor32);
        }
        Eold[b] = E;
        if (ok || bd || j + 1 == niter) {
          res[b].e0 = E;
          res[b].beta_last = tb[j + 1];
          res[b].iters = j + 1;
          res[b].status = (ok || bd) ? EDX_OK : EDX_E_NOCONV;
          res[b].breakdown = bd ? 1 : 0;
          done[b] = 1;
          --left;
        }
      }
    }
    steps = upto;
  }
  return EDX_OK;
}

// w = H v for K sets of one shape on interleaved vectors (no scale, no
// partial sums kept): the product of edx_hv_multi
size_t multi_hv_workspace_bytes(const edx_sector* s, int K, int vtype) {
  const size_t vb = align_up((size_t)s->vlen * K * vbytes(vtype));
  return multi_layout(s, K, vtype, 1, nullptr).total - 3 * vb + 256;
}

edx_status multi_hv(const edx_sector* const* secs, int K, int vtype, const void* v, void* w,
                    void* ws, size_t ws_bytes, hipStream_t st) {
  EDX_TRY(check_group(secs, K, vtype));
  const edx_sector* s0 = secs[0];
  char* base = reinterpret_cast<char*>(align_up(reinterpret_cast<uintptr_t>(ws)));
  // the layout without the Krylov vectors: tables and partial sums only
  MultiWs M = multi_layout(s0, K, vtype, 1, base);
  const size_t vb = align_up((size_t)s0->vlen * K * vbytes(vtype));
  const size_t shift = 3 * vb;
  if (M.total - shift + (size_t)(base - (char*)ws) > ws_bytes) {
    set_error("multi: workspace too small");
    return EDX_E_NOMEM;
  }
  M.amp -= shift;
  M.W -= shift;
  M.eup -= shift;
  M.edw -= shift;
  M.partial = (double*)((char*)M.partial - shift);
  EDX_TRY(stage_tables(secs, K, vtype, M, st));
  const uint32_t vbytes32 = (uint32_t)((uint64_t)s0->vlen * K * vbytes(vtype));
  if (vtype == EDX_F32) {
    MultiArgs<float> a{s0->dup, s0->ddw, s0->ld, s0->dw.hop, s0->hrow, s0->up.pat, s0->dw.pat,
                       (const float*)M.amp, (const float*)M.W, (const float*)M.eup,
                       (const float*)M.edw};
    return launch_multi<float>(a, K, s0->up.wpad, s0->dw.wpad, (const float*)v, (float*)w,
                               nullptr, M.partial, M.pstride, vbytes32, st);
  }
  MultiArgs<double> a{s0->dup, s0->ddw, s0->ld, s0->dw.hop, s0->hrow, s0->up.pat, s0->dw.pat,
                      (const double*)M.amp, (const double*)M.W, (const double*)M.eup,
                      (const double*)M.edw};
  return launch_multi<double>(a, K, s0->up.wpad, s0->dw.wpad, (const double*)v, (double*)w,
                              nullptr, M.partial, M.pstride, vbytes32, st);
}

}  // namespace edx
