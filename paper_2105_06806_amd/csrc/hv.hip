// Storage-free H.v for one sector (Sec. 3 "Matrix-vector product", eq. Hbuild).
//
// With v viewed as the D_up x D_dw column-major matrix V of eq. Vmatrix,
//   W = H_d o V + H_up V + V H_dw^T.
// The spin-up hops stay inside a column (contiguous), the spin-down hops stay
// inside a row (stride D_up).  The paper makes the row access local with an MPI
// transpose (Sec. 3.2).  One GPU holds the whole vector, so instead:
//
//  * k_hv_fused -- one pass: a block owns a group of consecutive columns,
//                 staged in LDS, so the spin-up gathers hit LDS; adds H_d and
//                 gathers the spin-down neighbours of each element straight
//                 from global memory (whole neighbour columns, coalesced).
//  * k_hv_col  -- the column pass of the two-pass plan: as k_hv_fused without
//                 the spin-down gathers, accumulating into w.
//  * k_hv_row  -- spin-down part over slabs of R consecutive rows.  A wave
//                 reads R contiguous elements of each neighbour column.  Blocks
//                 are numbered so that the blocks of one slab run on one XCD
//                 (workgroups go round-robin over the 8 XCDs), so the slab
//                 (R x D_dw elements) stays in that XCD's L2 while its ~8 reads
//                 per element are served.
//  * k_hv_small -- whole sector in LDS, one block (tiny sectors).
//
// Two-pass order: k_hv_row writes W = V H_dw^T, then k_hv_col adds
// H_d o V + H_up V in place and (optionally) the per-block partial sums of
// <v, w> needed by Lanczos.
//
// Column stride: V may be stored with a leading dimension ld >= D_up (the
// padding rows are neither read nor written).  With ld a multiple of 32
// elements every column starts on a 128-byte line, so a wave's 256-byte
// gather from a neighbour column touches two lines instead of three; the
// gathers are what bounds these kernels (load bandwidth between L2 and the
// CUs), so the Krylov vectors of the library use such an ld.
#include <algorithm>
#include <cmath>
#include <type_traits>
#include <vector>

#include "common.h"
#include "edx_internal.h"

namespace edx {

template <typename T>
struct HvArgs {
  int64_t dup, ddw;
  int64_t ld;                         // vector column stride (elements), >= dup
  const uint32_t* __restrict__ hup;   // row-major, stride sup
  const uint32_t* __restrict__ hdw;   // row-major, stride sdw
  int sup, sdw;                       // padded row lengths (8, 16 or 24)
  const T* __restrict__ eup;
  const T* __restrict__ edw;
  const uint8_t* __restrict__ pup;
  const uint8_t* __restrict__ pdw;
  const T* __restrict__ amp;   // [256]
  const T* __restrict__ W;     // [64]
  const uint8_t* __restrict__ hrow;   // compact spin-up rows (fused pass) or nullptr
};

template <typename T>
HvArgs<T> make_args(const edx_sector* s, int64_t ld);

template <>
HvArgs<double> make_args<double>(const edx_sector* s, int64_t ld) {
  return HvArgs<double>{s->dup, s->ddw, ld, s->up.hop, s->dw.hop, s->up.wpad, s->dw.wpad,
                        s->up.e64, s->dw.e64, s->up.pat, s->dw.pat, s->amp64, s->w64,
                        s->hrow};
}
template <>
HvArgs<float> make_args<float>(const edx_sector* s, int64_t ld) {
  return HvArgs<float>{s->dup, s->ddw, ld, s->up.hop, s->dw.hop, s->up.wpad, s->dw.wpad,
                       s->up.e32, s->dw.e32, s->up.pat, s->dw.pat, s->amp32, s->w32,
                       s->hrow};
}

// ---------------------------------------------------------------- small
template <typename T>
__global__ __launch_bounds__(1024) void k_hv_small(HvArgs<T> a, const T* __restrict__ v,
                                                   T* __restrict__ w,
                                                   const double* __restrict__ vscale,
                                                   double* __restrict__ partial) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* amp = reinterpret_cast<T*>(smem_raw);
  T* Wt = amp + kAmpTable;
  double* red = reinterpret_cast<double*>(Wt + 64);
  T* vs = reinterpret_cast<T*>(red + 16);
  const int64_t D = a.dup * a.ddw;
  const T sc = vscale ? (T)(*vscale) : T(1);
  for (int i = threadIdx.x; i < kAmpTable; i += blockDim.x) amp[i] = a.amp[i];
  for (int i = threadIdx.x; i < 64; i += blockDim.x) Wt[i] = a.W[i];
  for (int64_t i = threadIdx.x; i < D; i += blockDim.x)
    vs[i] = v[i % a.dup + (i / a.dup) * a.ld] * sc;
  __syncthreads();
  double dot = 0.0;
  for (int64_t idx = threadIdx.x; idx < D; idx += blockDim.x) {
    const int64_t iu = idx % a.dup;
    const int64_t id = idx / a.dup;
    const T x = vs[idx];
    T acc = (a.eup[iu] + a.edw[id] + Wt[a.pup[iu] * 8 + a.pdw[id]]) * x;
    for (int k = 0; k < a.sup; ++k) {
      const uint32_t e = a.hup[iu * a.sup + k];
      acc += amp[e >> kAmpShift] * vs[id * a.dup + (e & kColMask)];
    }
    for (int k = 0; k < a.sdw; ++k) {
      const uint32_t e = a.hdw[id * a.sdw + k];
      acc += amp[e >> kAmpShift] * vs[iu + (int64_t)(e & kColMask) * a.dup];
    }
    w[iu + id * a.ld] = acc;
    dot += (double)x * (double)acc;
  }
  const int64_t pad = a.ld - a.dup;
  for (int64_t i = threadIdx.x; i < pad * a.ddw; i += blockDim.x)
    w[a.dup + (i % pad) + (i / pad) * a.ld] = T(0);
  if (partial) {
    const double s = block_sum(dot, red);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
  }
}

// ---------------------------------------------------------------- column pass
// Latency hiding: the column staging issues 8 independent loads per thread
// before storing them; every row's whole (padded) hop list comes in with
// vector loads; the accumulate variant processes two rows per thread so that
// the table loads and the read of w for both are in flight together.
constexpr int kColMax = 4;   // columns per block held in registers per thread

// nc (<= kColMax) consecutive columns of dup elements, column stride ld, into
// a dense LDS image; the column of flat index i is found by comparisons.
template <typename T>
__device__ __forceinline__ void stage_cols(T* __restrict__ vs, const T* __restrict__ src, int nc,
                                           int64_t dup, int64_t ld, T sc) {
  const int64_t n = (int64_t)nc * dup;
  const int64_t gap = ld - dup;
  auto at = [&](int64_t i) {
    const int64_t c = (int64_t)(i >= dup) + (int64_t)(i >= 2 * dup) + (int64_t)(i >= 3 * dup);
    return src[i + c * gap];
  };
  const int bd = blockDim.x;
  int64_t i = threadIdx.x;
  for (; i + 7 * bd < n; i += 8 * bd) {
    T x[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) x[u] = at(i + u * bd);
#pragma unroll
    for (int u = 0; u < 8; ++u) vs[i + u * bd] = x[u] * sc;
  }
  for (; i < n; i += bd) vs[i] = at(i) * sc;
}

// BUF: the spin-down gathers are buffer loads (resource over v, vbytes bytes):
// each neighbour column's byte offset sits in a scalar register and every
// gather of a row shares one 32-bit lane offset, where a global load needs a
// 64-bit address per lane and gather.  Requires vbytes < 2^32.
template <typename T>
__device__ __forceinline__ T buf_load(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  if constexpr (sizeof(T) == 4) {
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, 0));
  } else {
    typedef unsigned int u2 __attribute__((ext_vector_type(2)));
    const u2 x = __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, (int)soff, 0);
    return __longlong_as_double((long long)(((unsigned long long)x.y << 32) | x.x));
  }
}

// the same with the non-temporal hint (the line is not kept for reuse)
template <typename T>
__device__ __forceinline__ T buf_load_nt(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  if constexpr (sizeof(T) == 4) {
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, 2));
  } else {
    typedef unsigned int u2 __attribute__((ext_vector_type(2)));
    const u2 x = __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, (int)soff, 2);
    return __longlong_as_double((long long)(((unsigned long long)x.y << 32) | x.x));
  }
}

// streaming (non-temporal) buffer store
template <typename T>
__device__ __forceinline__ void buf_store_nt(__amdgpu_buffer_rsrc_t r, uint32_t voff,
                                             uint32_t soff, T x) {
  if constexpr (sizeof(T) == 4) {
    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(x), r, (int)voff, (int)soff, 2);
  } else {
    typedef unsigned int u2 __attribute__((ext_vector_type(2)));
    const unsigned long long b = (unsigned long long)__double_as_longlong(x);
    u2 y;
    y.x = (unsigned)b;
    y.y = (unsigned)(b >> 32);
    __builtin_amdgcn_raw_buffer_store_b64(y, r, (int)voff, (int)soff, 2);
  }
}

// nc (<= NC) arbitrary columns jc[0..nc) of a vector with column stride ld
// into an interleaved LDS image: element r of column c at r * NC + c, so one
// spin-up hop reads the NC values it needs from adjacent words.  In passes of
// U rows per thread: stage_issue puts every load of a pass in flight (one
// memory latency per pass; for Ns = 16 FP32 and NC = 3 one pass covers the
// columns), stage_put scales and stores them, so the block-uniform set-up can
// run between the two.
template <typename T, int NC, int U>
struct StageBuf {
  T x[NC][U];
};

template <typename T, int NC, int U>
__device__ __forceinline__ void stage_issue(StageBuf<T, NC, U>& b, const T* __restrict__ v,
                                            const int64_t (&jc)[NC], int nc, int64_t dup,
                                            int64_t ld, int64_t r0) {
  const int bd = blockDim.x;
#pragma unroll
  for (int c = 0; c < NC; ++c)
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t r = r0 + (int64_t)u * bd;
      b.x[c][u] = (c < nc && r < dup) ? v[jc[c] * ld + r] : T(0);
    }
}

// the same through a buffer resource over v: one 32-bit lane offset per row,
// the column offsets (coff, bytes) block-uniform
// The workgroup's own columns are read once here and next needed only as
// spin-down neighbours of other columns, long after they would have left L2.
// FP32: a non-temporal load keeps them from displacing neighbour lines that
// concurrently running workgroups share (Ns=16 8/8, 3 columns: 726 -> 706 us).
// FP64 keeps the default policy (non-temporal there: 1702 -> 1750 us).
template <typename T>
__device__ __forceinline__ T stage_load(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  if constexpr (sizeof(T) == 4)
    return buf_load_nt<T>(r, voff, soff);
  else
    return buf_load<T>(r, voff, soff);
}

template <typename T, int NC, int U>
__device__ __forceinline__ void stage_issue_buf(StageBuf<T, NC, U>& b, __amdgpu_buffer_rsrc_t r,
                                                const uint32_t (&coff)[NC], int nc, uint32_t dup,
                                                uint32_t r0) {
  const uint32_t bd = blockDim.x;
#pragma unroll
  for (int c = 0; c < NC; ++c)
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint32_t row = r0 + (uint32_t)u * bd;
      b.x[c][u] = (c < nc && row < dup) ? stage_load<T>(r, row * (uint32_t)sizeof(T), coff[c])
                                        : T(0);
    }
}

template <typename T, int NC, int U>
__device__ __forceinline__ void stage_put(T* __restrict__ vs, const StageBuf<T, NC, U>& b, int nc,
                                          int64_t dup, int64_t r0, T sc) {
  const int bd = blockDim.x;
#pragma unroll
  for (int c = 0; c < NC; ++c)
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t r = r0 + (int64_t)u * bd;
      if (c < nc && r < dup) vs[r * NC + c] = b.x[c][u] * sc;
    }
}

template <int W>
__device__ __forceinline__ void load_row(const uint32_t* __restrict__ h, int64_t i,
                                         uint32_t (&e)[W]) {
  const uint4* ep = reinterpret_cast<const uint4*>(h + i * W);
#pragma unroll
  for (int q = 0; q < W / 4; ++q) {
    const uint4 x = ep[q];
    e[4 * q] = x.x; e[4 * q + 1] = x.y; e[4 * q + 2] = x.z; e[4 * q + 3] = x.w;
  }
}

// Column pass of the two-pass plan: w += H_d o V + H_up V (w holds V H_dw^T).
template <typename T, int WUP>
__global__ __launch_bounds__(1024) void k_hv_col(HvArgs<T> a, const T* __restrict__ v,
                                                 T* __restrict__ w,
                                                 const double* __restrict__ vscale,
                                                 double* __restrict__ partial, int ncol,
                                                 int accumulate) {
  constexpr int RPT = 2;   // rows per thread per iteration
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* amp = reinterpret_cast<T*>(smem_raw);
  T* Wt = amp + kAmpTable;
  double* red = reinterpret_cast<double*>(Wt + 64);
  T* vs = reinterpret_cast<T*>(red + 16);
  const int64_t dup = a.dup;
  const int64_t j0 = (int64_t)blockIdx.x * ncol;
  const int nc = (int)std::min<int64_t>(ncol, a.ddw - j0);
  const T sc = vscale ? (T)(*vscale) : T(1);
  for (int i = threadIdx.x; i < kAmpTable; i += blockDim.x) amp[i] = a.amp[i];
  for (int i = threadIdx.x; i < 64; i += blockDim.x) Wt[i] = a.W[i];
  const int64_t ld = a.ld;
  stage_cols(vs, v + j0 * ld, nc, dup, ld, sc);
  __syncthreads();
  int64_t jc[kColMax];
  T ed[kColMax];
  int pd[kColMax];
#pragma unroll
  for (int c = 0; c < kColMax; ++c) {
    jc[c] = j0 + (c < nc ? c : 0);
    ed[c] = a.edw[jc[c]];
    pd[c] = a.pdw[jc[c]];
  }
  double dot = 0.0;
  for (int64_t base = threadIdx.x; base < dup; base += RPT * blockDim.x) {
    int64_t rows[RPT];
    bool ok[RPT];
    uint32_t e[RPT][WUP];
    T eu[RPT];
    int pu[RPT];
    T wold[RPT][kColMax];
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
      const int64_t iu = base + (int64_t)r * blockDim.x;
      ok[r] = iu < dup;
      rows[r] = ok[r] ? iu : base;
      load_row<WUP>(a.hup, rows[r], e[r]);
      eu[r] = a.eup[rows[r]];
      pu[r] = a.pup[rows[r]] * 8;
#pragma unroll
      for (int c = 0; c < kColMax; ++c)
        wold[r][c] = (c < nc && accumulate) ? w[rows[r] + jc[c] * ld] : T(0);
    }
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
      if (!ok[r]) continue;
      const int64_t iu = rows[r];
      T acc[kColMax];
#pragma unroll
      for (int c = 0; c < kColMax; ++c) acc[c] = T(0);
#pragma unroll
      for (int k = 0; k < WUP; ++k) {
        const T am = amp[e[r][k] >> kAmpShift];
        const int64_t col = e[r][k] & kColMask;
#pragma unroll
        for (int c = 0; c < kColMax; ++c)
          if (c < nc) acc[c] += am * vs[c * dup + col];
      }
#pragma unroll
      for (int c = 0; c < kColMax; ++c) {
        if (c >= nc) break;
        const int64_t j = jc[c];
        const T x = vs[c * dup + iu];
        const T res = acc[c] + (eu[r] + ed[c] + Wt[pu[r] + pd[c]]) * x + wold[r][c];
        w[iu + j * ld] = res;
        dot += (double)x * (double)res;
      }
    }
  }
  // padding rows of the output are defined as zero
  for (int64_t i = dup + threadIdx.x; i < ld; i += blockDim.x)
    for (int c = 0; c < nc; ++c) w[i + (j0 + c) * ld] = T(0);
  if (partial) {
    const double s = block_sum(dot, red);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
  }
}

// ---------------------------------------------------------------- fused pass
// One pass: a block owns NC consecutive columns (staged in LDS); per row it
// issues the NC * WDW spin-down gathers from global memory first (their table
// rows, pre-scaled amplitudes and column offsets are block-uniform and loaded
// once), then does the spin-up hops from LDS and H_d while they are in flight.
// The last block may own fewer columns: it computes clamped copies and stores
// only its own.
// Block-uniform values forced into scalar registers.
__device__ __forceinline__ float uniform(float x) {
  return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(x)));
}
__device__ __forceinline__ double uniform(double x) {
  const long long b = __double_as_longlong(x);
  const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)b);
  const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(b >> 32));
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
// a pointer into global memory (address space 1: global, not flat, loads)
template <typename T>
using gptr = const T __attribute__((address_space(1)))*;
template <typename T>
__device__ __forceinline__ gptr<T> uniform(const T* p) {
  const unsigned long long b = reinterpret_cast<unsigned long long>(p);
  const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)b);
  const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(b >> 32));
  return (gptr<T>)(((unsigned long long)hi << 32) | lo);
}

// Spin-exchange / pair-hopping term table of a sector (see k_hv_nd): per
// impurity-pattern pair, the row and column shifts of the source element
// and the signed amplitude.
template <typename T>
struct NdTab {
  const int32_t* off;   // [P*P + 1]
  const int32_t* du;
  const int32_t* dd;
  const T* amp;
  int P, nt;
};

// terms of the fused pass's staged table: H_nd, or with phonons the largest
// per-slice table (H_nd + phonon terms)
inline int nd_lds_terms(const edx_sector* s) {
  if (!s->nd) return 0;   // phonons alone use the direct path, no table
  return s->dph > 1 ? s->ph_nt_max : s->nd_nt;
}

template <typename T>
const T* ph_amp(const edx_sector* s);
template <>
const double* ph_amp<double>(const edx_sector* s) { return s->ph_amp64; }
template <>
const float* ph_amp<float>(const edx_sector* s) { return s->ph_amp32; }
template <typename T>
const T* wph(const edx_sector* s);
template <>
const double* wph<double>(const edx_sector* s) { return s->wph64; }
template <>
const float* wph<float>(const edx_sector* s) { return s->wph32; }

// Holstein terms of one phonon slice p for the fused pass (Sec. "Electron-phonon
// coupling"): (g(pu) + g(pd)) (sp v_{p-1} + sp1 v_{p+1}) at the element itself,
// the neighbouring slices `slice` elements away; g(pattern) = sum_a g_a n_a.
template <typename T>
struct PhArgs {
  int64_t slice;   // elements per phonon slice (ld * D_dw)
  T sp, sp1;       // sqrt(p), sqrt(p + 1)
  T g0, g1, g2;    // couplings g_a
  int lo, hi;      // slice p - 1 / p + 1 exists
};

template <typename T>
__device__ __forceinline__ T gpat(const PhArgs<T>& ph, int pat) {
  return ((pat & 1) ? ph.g0 : T(0)) + ((pat & 2) ? ph.g1 : T(0)) + ((pat & 4) ? ph.g2 : T(0));
}

template <typename T>
const T* nd_amp(const edx_sector* s);
template <>
const double* nd_amp<double>(const edx_sector* s) { return s->nd_amp64; }
template <>
const float* nd_amp<float>(const edx_sector* s) { return s->nd_amp32; }

__host__ __device__ constexpr size_t al16(size_t x) { return (x + 15) & ~(size_t)15; }

// LDS bytes of a staged term table
inline size_t nd_tab_lds(int P, int nt, size_t tsz) {
  return al16((size_t)(P * P + 1) * 4) + al16((size_t)nt * 8) + al16((size_t)nt * tsz);
}

constexpr int64_t kWinGroups = 32;   // column groups per XCD in a window (its CUs)

template <typename T, int WUP, int WDW, int NC, bool ND, bool PH, bool BUF>
__global__ __launch_bounds__(1024) void k_hv_fused(HvArgs<T> a, const T* __restrict__ v,
                                                   T* __restrict__ w,
                                                   const double* __restrict__ vscale,
                                                   double* __restrict__ partial, int order,
                                                   const int32_t* __restrict__ corder,
                                                   NdTab<T> nd, PhArgs<T> ph, uint32_t vbytes) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  // LDS: the staged columns first (at offset 0, so a spin-up hop's address is
  // a single multiply), then the amplitude and W tables and the reduction slots
  T* vs = reinterpret_cast<T*>(smem_raw);
  T* amp = reinterpret_cast<T*>(smem_raw + al16((size_t)NC * a.dup * sizeof(T)));
  T* Wt = amp + kAmpTable;
  double* red = reinterpret_cast<double*>(Wt + 64);
  const int64_t dup = a.dup, ld = a.ld;
  // with ND the spin-exchange / pair-hopping table follows the columns:
  // offsets, (row shift, column shift) pairs, amplitudes
  int* n_off = nullptr;
  int2* n_dud = nullptr;
  T* n_amp = nullptr;
  if (ND) {
    unsigned char* q = reinterpret_cast<unsigned char*>(red + 16);
    n_off = reinterpret_cast<int*>(q);
    n_dud = reinterpret_cast<int2*>(q + al16((size_t)(nd.P * nd.P + 1) * 4));
    n_amp = reinterpret_cast<T*>(reinterpret_cast<unsigned char*>(n_dud) +
                                 al16((size_t)nd.nt * 8));
    for (int k = threadIdx.x; k <= nd.P * nd.P; k += blockDim.x) n_off[k] = nd.off[k];
    for (int k = threadIdx.x; k < nd.nt; k += blockDim.x) {
      n_dud[k] = make_int2(nd.du[k], nd.dd[k]);
      n_amp[k] = nd.amp[k];
    }
  }
  // Which columns: group cb = workgroup index (order 0), or XCD-contiguous
  // numbering (orders 1 and 2): workgroups go round-robin over the 8 XCDs, so
  // workgroup b takes group x*q + min(x, r) + b/8 (x = b % 8) and the groups
  // running at once on one XCD are consecutive; their spin-down neighbours
  // overlap and are served by that XCD's L2.  Orders 3 and 4: the same inside
  // windows that all XCDs walk together.  Orders 2 and 4 walk the columns
  // sorted by impurity occupation, where consecutive columns share more
  // neighbours.
  int64_t cb = blockIdx.x;
  if (order == 1 || order == 2) {
    const int64_t nblk = gridDim.x, q8 = nblk / 8, r8 = nblk % 8;
    const int64_t x8 = blockIdx.x % 8;
    cb = x8 * q8 + std::min<int64_t>(x8, r8) + blockIdx.x / 8;
  } else if (order >= 3) {
    // windows of 8 * wg consecutive groups (wg = 32, one per CU, over the
    // columns in listing order; 64 over the sorted columns -- the measured
    // best): inside a window XCD x takes the groups x*wg ... x*wg + wg - 1,
    // so the groups resident on one XCD are consecutive (their neighbours
    // meet in its L2) and all XCDs work in the same window (its neighbour
    // columns meet in the MALL); the last, partial window keeps the
    // workgroup order
    const int64_t wg = order == 3 ? kWinGroups : 2 * kWinGroups;
    const int64_t win = 8 * wg;
    const int64_t b = blockIdx.x, w0 = b - b % win;
    if (w0 + win <= (int64_t)gridDim.x) {
      const int64_t r = b - w0;
      cb = w0 + (r % 8) * wg + r / 8;
    }
  }
  const int64_t j0 = cb * NC;
  const int nc = (int)std::min<int64_t>(NC, a.ddw - j0);
  int64_t jc[NC];   // this workgroup's columns (clamped copies past the end)
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const int64_t jj = std::min<int64_t>(j0 + c, a.ddw - 1);
    jc[c] = (order == 2 || order == 4) ? (int64_t)__builtin_amdgcn_readfirstlane(corder[jj]) : jj;
  }
  const T sc = vscale ? (T)(*vscale) : T(1);
  // first staging pass in flight while the tables and the block-uniform
  // neighbour set-up are loaded
  // rows per thread per staging pass (BUF: 40 FP32 / 20 FP64 loads in flight;
  // otherwise as many as leave the larger ND / PH bodies without spills)
  constexpr int SU = BUF ? std::max(1, (sizeof(T) == 4 ? 40 : 20) / NC)
                         : (NC >= 3 ? 4 : 8 / NC);
  StageBuf<T, NC, SU> sb;
  __amdgpu_buffer_rsrc_t vres;
  uint32_t coff[NC];   // BUF: byte offsets of the block's columns
  if constexpr (BUF) {
    vres = __builtin_amdgcn_make_buffer_rsrc(const_cast<T*>(v), 0, (int)vbytes, 0x00020000);
#pragma unroll
    for (int c = 0; c < NC; ++c)
      coff[c] = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)jc[c] * ld * sizeof(T)));
    stage_issue_buf(sb, vres, coff, nc, (uint32_t)dup, threadIdx.x);
  } else {
    stage_issue(sb, v, jc, nc, dup, ld, (int64_t)threadIdx.x);
  }
  for (int i = threadIdx.x; i < kAmpTable; i += blockDim.x) amp[i] = a.amp[i];
  for (int i = threadIdx.x; i < 64; i += blockDim.x) Wt[i] = a.W[i];
  gptr<T> gcol[NC][WDW];   // neighbour columns (block-uniform)
  uint32_t goff[NC][WDW];  // BUF: their byte offsets from v
  T gamp[NC][WDW];         // their amplitudes times the vector scale
  int nreal[NC];           // real (not padding) entries of the column's hop row
  T ed[NC];
  int pd[NC];
  T gd[NC];   // phonon coupling of the spin-down pattern (PH)
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const int64_t j = jc[c];
    ed[c] = a.edw[j];
    pd[c] = a.pdw[j];
    gd[c] = PH ? gpat(ph, pd[c]) : T(0);
    int cnt = 0;
#pragma unroll
    for (int k = 0; k < WDW; ++k) {
      const uint32_t f = a.hdw[j * WDW + k];
      cnt += (f >> kAmpShift) != kPadPair ? 1 : 0;
      if constexpr (BUF)
        goff[c][k] = __builtin_amdgcn_readfirstlane(
            (uint32_t)((uint64_t)(f & kColMask) * (uint64_t)ld * sizeof(T)));
      else
        gcol[c][k] = uniform(v + (int64_t)(f & kColMask) * ld);
      gamp[c][k] = uniform(a.amp[f >> kAmpShift] * sc);
    }
    nreal[c] = (int)__builtin_amdgcn_readfirstlane((uint32_t)cnt);
  }
  stage_put(vs, sb, nc, dup, (int64_t)threadIdx.x, sc);
  for (int64_t r0 = threadIdx.x + (int64_t)SU * blockDim.x; r0 < dup;
       r0 += (int64_t)SU * blockDim.x) {
    if constexpr (BUF)
      stage_issue_buf(sb, vres, coff, nc, (uint32_t)dup, (uint32_t)r0);
    else
      stage_issue(sb, v, jc, nc, dup, ld, r0);
    stage_put(vs, sb, nc, dup, r0, sc);
  }
  // BUF: buffer resources over v, w and the row tables; every row offset is
  // 32-bit and the store offsets of the NC output columns are block-uniform
  constexpr int HW = 3 * WUP / 4;   // 32-bit words of a compact spin-up row
  __amdgpu_buffer_rsrc_t wres, hres, eres, pres;
  uint32_t woff[NC];
  if constexpr (BUF) {
    wres = __builtin_amdgcn_make_buffer_rsrc(w, 0, (int)vbytes, 0x00020000);
    hres = __builtin_amdgcn_make_buffer_rsrc(const_cast<uint8_t*>(a.hrow), 0,
                                             (int)(dup * HW * 4), 0x00020000);
    eres = __builtin_amdgcn_make_buffer_rsrc(const_cast<T*>(a.eup), 0, (int)(dup * sizeof(T)),
                                             0x00020000);
    pres = __builtin_amdgcn_make_buffer_rsrc(const_cast<uint8_t*>(a.pup), 0, (int)dup,
                                             0x00020000);
#pragma unroll
    for (int c = 0; c < NC; ++c) woff[c] = coff[c];
  }
  __syncthreads();
  double dot = 0.0;
  // ALL: the block owns NC columns (every block but possibly the last); then
  // nothing in the row body is conditional and the compiler keeps all
  // gathers of a row in flight together
  // WK: spin-down slots gathered per row -- 8 when no column of the block has
  // more real hops than that (the padding entries follow the real ones), else
  // every slot of the padded row
  auto rows = [&](auto all_tag, auto wk_tag) {
    constexpr bool ALL = decltype(all_tag)::value;
    constexpr int WK = decltype(wk_tag)::value;
    // (BUF: a 32-bit row index; D_up < 2^24 always)
    using RowT = std::conditional_t<BUF, uint32_t, int64_t>;
    for (RowT iu = threadIdx.x; iu < (RowT)dup; iu += blockDim.x) {
      // the row's own tables first: loads complete in issue order, so the
      // spin-up part can start before the gathers have arrived
      const uint32_t iu32 = (uint32_t)iu;
      const uint32_t voff = iu32 * (uint32_t)sizeof(T);
      // hop k: column col[k] (bits 0..23 of e[k]), amplitude index ai[k]
      uint32_t e[WUP];
      uint32_t col[WUP], ai[WUP];
      T eu;
      int patu;
      if constexpr (BUF) {
        // compact row: 16-bit columns, then 8-bit amplitude indices
        uint32_t r[HW];
#pragma unroll
        for (int q = 0; q < HW / 2; ++q) {
          typedef unsigned int u2 __attribute__((ext_vector_type(2)));
          const u2 x = __builtin_amdgcn_raw_buffer_load_b64(hres, (int)(iu32 * HW * 4 + q * 8),
                                                            0, 0);
          r[2 * q] = x.x;
          r[2 * q + 1] = x.y;
        }
        eu = buf_load<T>(eres, voff, 0);
        patu = __builtin_amdgcn_raw_buffer_load_b8(pres, (int)iu32, 0, 0);
#pragma unroll
        for (int k = 0; k < WUP; ++k) {
          col[k] = (r[k >> 1] >> (16 * (k & 1))) & 0xFFFFu;
          ai[k] = (r[WUP / 2 + (k >> 2)] >> (8 * (k & 3))) & 0xFFu;
        }
      } else {
        load_row<WUP>(a.hup, iu, e);
        eu = a.eup[iu];
        patu = a.pup[iu];
#pragma unroll
        for (int k = 0; k < WUP; ++k) {
          col[k] = e[k] & kColMask;
          ai[k] = e[k] >> kAmpShift;
        }
      }
      const int pu = patu * 8;
      T g[NC][WDW];
#pragma unroll
      for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int k = 0; k < WK; ++k) {
          if constexpr (BUF) {
            if constexpr (WK > 8 && sizeof(T) == 8) {
              // the full-width loop over padded hop rows (Norb >= 2: 16
              // slots, 6.4-7.5 real hops on average at Ns = 15-16): the
              // padding entries come after the real ones and carry amplitude
              // 0, so in FP64 a block-uniform branch skips their loads
              // (Norb=2 Ns=16 3100 -> 2074 us, Norb=3 Ns=15 537 -> 459 us);
              // FP32 keeps every load of the row in one batch (the branches
              // cost it 4-24 %).
              if (k < nreal[c])
                g[c][k] = buf_load<T>(vres, voff, goff[c][k]);
              else
                g[c][k] = T(0);
            } else {
              g[c][k] = buf_load<T>(vres, voff, goff[c][k]);
            }
          } else {
            g[c][k] = gcol[c][k][iu32];
          }
        }
      // phonon neighbours: the same element one slice back / ahead, issued
      // with the gathers so that their latency overlaps
      T pv[NC], pn[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        pv[c] = T(0);
        pn[c] = T(0);
        if constexpr (PH) {
          const int64_t e0 = iu + jc[c] * ld;
          if (ph.lo) pv[c] = v[e0 - ph.slice];
          if (ph.hi) pn[c] = v[e0 + ph.slice];
        }
      }
      T acc[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) acc[c] = T(0);
#pragma unroll
      for (int k = 0; k < WUP; ++k) {
        const T ak = amp[ai[k]];
        const T* src = vs + __umul24(col[k], (uint32_t)NC);
#pragma unroll
        for (int c = 0; c < NC; ++c) acc[c] += ak * src[c];
      }
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        const T x = vs[iu32 * (uint32_t)NC + c];
        T s2 = T(0);
#pragma unroll
        for (int k = 0; k < WK; ++k) s2 += gamp[c][k] * g[c][k];
        T res = acc[c] + (eu + ed[c] + Wt[pu + pd[c]]) * x + s2;
        if constexpr (PH) res += (gpat(ph, patu) + gd[c]) * (ph.sp * pv[c] + ph.sp1 * pn[c]) * sc;
        if constexpr (ND) {
          // spin exchange / pair hopping: sources near (iu, jc[c])
          const int key = patu * nd.P + pd[c];
          const int t1 = n_off[key + 1];
          T sn = T(0);
          for (int t = n_off[key]; t < t1; ++t) {
            const int2 sh = n_dud[t];
            sn += n_amp[t] * v[iu + sh.x + (jc[c] + sh.y) * ld];
          }
          res += sn * sc;
        }
        if (ALL || c < nc) {
          // streaming store: w is not read again in this pass, so it should
          // not displace the neighbour columns the gathers reuse from L2
          if constexpr (BUF)
            buf_store_nt<T>(wres, voff, woff[c], res);
          else
            __builtin_nontemporal_store(res, &w[iu + jc[c] * ld]);
          dot += (double)x * (double)res;
        }
      }
    }
  };
  // Padded rows of 16 slots (Norb >= 2): 80-93 % of the blocks have no column
  // with more than 8 real hops (Norb=2 Ns=16, 3 columns: 80 %; Norb=3 Ns=15,
  // 2 columns: 86 %), and those take a row loop over 8 slots.  Measured: FP32
  // Norb=2 Ns=16 1169 -> 1038 us, Norb=3 Ns=15 235 -> 217 us; FP64 with 2
  // columns a block Norb=3 Ns=15 467 -> 412 us.  FP64 with one column a block
  // keeps the per-load skip alone (the 8-slot loop was 4 % slower there).
  constexpr bool kNarrow = WDW > 8 && (sizeof(T) == 4 || NC >= 2);
  bool narrow = false;
  if constexpr (kNarrow) {
    int mx = 0;
#pragma unroll
    for (int c = 0; c < NC; ++c) mx = std::max(mx, nreal[c]);
    narrow = mx <= 8;
  }
  auto go = [&](auto all_tag) {
    if constexpr (kNarrow) {
      if (narrow)
        rows(all_tag, std::integral_constant<int, 8>{});
      else
        rows(all_tag, std::integral_constant<int, WDW>{});
    } else {
      rows(all_tag, std::integral_constant<int, WDW>{});
    }
  };
  if (nc == NC)
    go(std::true_type{});
  else
    go(std::false_type{});
  for (int64_t i = dup + threadIdx.x; i < ld; i += blockDim.x)
#pragma unroll
    for (int c = 0; c < NC; ++c)
      if (c < nc) w[i + jc[c] * ld] = T(0);
  if (partial) {
    const double s = block_sum(dot, red);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
  }
}

// ---------------------------------------------------------------- row pass
// A wave covers R*VEC consecutive rows (VEC rows per lane, one vector load) of
// 64/R columns; each thread handles two columns per iteration with all their
// gathers in flight.
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef double f64x2 __attribute__((ext_vector_type(2)));
template <typename T, int VEC>
struct VecT;
template <> struct VecT<float, 1> { using type = float; };
template <> struct VecT<float, 2> { using type = f32x2; };
template <> struct VecT<double, 1> { using type = double; };
template <> struct VecT<double, 2> { using type = f64x2; };

template <typename T, int R, int VEC, int WDW>
__global__ __launch_bounds__(256) void k_hv_row(HvArgs<T> a, const T* __restrict__ v,
                                                T* __restrict__ w,
                                                const double* __restrict__ vscale,
                                                int64_t nchunk, int cpb, int64_t nwork) {
  using V = typename VecT<T, VEC>::type;
  __shared__ T amp[kAmpTable];
  for (int i = threadIdx.x; i < kAmpTable; i += blockDim.x) amp[i] = a.amp[i];
  __syncthreads();
  // XCD-aware numbering: block b runs on XCD b % 8; give each XCD a contiguous
  // range of work items so that concurrently resident blocks share a slab.
  const int64_t b = blockIdx.x;
  const int64_t q = (nwork + 7) >> 3;
  const int64_t work = (b & 7) * q + (b >> 3);
  if (work >= nwork) return;
  const int64_t slab = work / nchunk;
  const int64_t chunk = work - slab * nchunk;
  const int r = threadIdx.x % R;
  const int cw = threadIdx.x / R;
  constexpr int kColsInFlight = 256 / R;
  const int64_t iu = (slab * R + r) * VEC;        // first row of this lane
  const bool ok = iu < a.dup;                     // VEC = 2 needs an even D_up
  const int64_t iuc = ok ? iu : 0;
  const T sc = vscale ? (T)(*vscale) : T(1);
  const int64_t jb = chunk * cpb;
  const int64_t je = std::min<int64_t>(jb + cpb, a.ddw);
  for (int64_t j = jb + cw; j < je; j += 2 * kColsInFlight) {
    const int64_t j2 = j + kColsInFlight;
    const bool has2 = j2 < je;
    const int64_t j2c = has2 ? j2 : j;
    // with R = 64 a wave covers one column, so the table row is wave-uniform
    // and goes through the scalar cache
    const int64_t ja = R == 64 ? (int64_t)__builtin_amdgcn_readfirstlane((int)j) : j;
    const int64_t jb2 = R == 64 ? (int64_t)__builtin_amdgcn_readfirstlane((int)j2c) : j2c;
    uint32_t e1[WDW], e2[WDW];
#pragma unroll
    for (int k = 0; k < WDW; ++k) {
      e1[k] = a.hdw[ja * WDW + k];
      e2[k] = a.hdw[jb2 * WDW + k];
    }
    V g1[WDW], g2[WDW];
#pragma unroll
    for (int k = 0; k < WDW; ++k) {
      g1[k] = *reinterpret_cast<const V*>(v + iuc + (int64_t)(e1[k] & kColMask) * a.ld);
      g2[k] = *reinterpret_cast<const V*>(v + iuc + (int64_t)(e2[k] & kColMask) * a.ld);
    }
    V s1 = V(0), s2 = V(0);
#pragma unroll
    for (int k = 0; k < WDW; ++k) {
      s1 += (amp[e1[k] >> kAmpShift] * sc) * g1[k];
      s2 += (amp[e2[k] >> kAmpShift] * sc) * g2[k];
    }
    // streaming stores: keep L2 for the slab being gathered
    if (ok) {
      __builtin_nontemporal_store(s1, reinterpret_cast<V*>(w + iu + j * a.ld));
      if (has2) __builtin_nontemporal_store(s2, reinterpret_cast<V*>(w + iu + j2 * a.ld));
    }
  }
}

// ---------------------------------------------------------------- H_nd pass
// Spin exchange and pair hopping of eq. Ham1 (impurity orbitals p != q) move
// electrons of both spins at once, so they are no Kronecker sum: this pass
// adds them to w after the spin-separable passes.  H is real symmetric, so
// row i of these terms is the operators applied to |i>; whether a term acts,
// its sign and the index shift of the source element depend only on the
// impurity patterns of the row and column strings (the sector build tabulates
// them per pattern pair, see tables.hip), so an output element reads its
// row's pattern byte and gathers one nearby source element per term.
template <typename T>
struct NdArgs {
  int64_t dup, ddw, ld;
  const uint8_t* __restrict__ pup;
  const uint8_t* __restrict__ pdw;
  const int32_t* __restrict__ off;   // [P*P + 1]
  const int32_t* __restrict__ du;
  const int32_t* __restrict__ dd;
  const T* __restrict__ amp;
  int P;
};

constexpr int kNdMaxTerms = 64 * 12;   // pattern pairs (norb <= 3) x terms per pair
constexpr int kNdRows = 4;             // rows per thread per iteration (loads in flight)
constexpr int64_t kNdPatLds = 96 * 1024;   // row patterns staged in LDS up to this many rows

// The term table and (when D_up <= kNdPatLds) every row's impurity pattern
// are staged in LDS, so the only global loads left are the source gathers
// and the read-modify-write of w, issued together.
template <typename T>
__global__ __launch_bounds__(256) void k_hv_nd(NdArgs<T> a, const T* __restrict__ v,
                                               T* __restrict__ w,
                                               const double* __restrict__ vscale,
                                               double* __restrict__ partial) {
  __shared__ double red[16];
  __shared__ int s_off[65];
  __shared__ int s_du[kNdMaxTerms];
  __shared__ int s_dd[kNdMaxTerms];
  __shared__ T s_amp[kNdMaxTerms];
  extern __shared__ uint8_t s_pat[];
  const bool pat_lds = a.dup <= kNdPatLds;
  const int npp = a.P * a.P;
  for (int k = threadIdx.x; k <= npp; k += blockDim.x) s_off[k] = a.off[k];
  if (pat_lds)
    for (int64_t i = threadIdx.x; i < a.dup; i += blockDim.x) s_pat[i] = a.pup[i];
  __syncthreads();
  const int nt = s_off[npp];
  for (int k = threadIdx.x; k < nt; k += blockDim.x) {
    s_du[k] = a.du[k];
    s_dd[k] = a.dd[k];
    s_amp[k] = a.amp[k];
  }
  __syncthreads();
  const T sc = vscale ? (T)(*vscale) : T(1);
  double dot = 0.0;
  const int64_t step = (int64_t)blockDim.x * kNdRows;
  for (int64_t j = blockIdx.x; j < a.ddw; j += gridDim.x) {
    const int pd = a.pdw[j];
    const T* __restrict__ vcol = v + j * a.ld;
    T* __restrict__ wcol = w + j * a.ld;
    for (int64_t i0 = threadIdx.x; i0 < a.dup; i0 += step) {
      int t0[kNdRows], t1[kNdRows];
      T wold[kNdRows];
#pragma unroll
      for (int r = 0; r < kNdRows; ++r) {
        const int64_t i = i0 + (int64_t)r * blockDim.x;
        t0[r] = t1[r] = 0;
        if (i < a.dup) {
          const int key = (pat_lds ? (int)s_pat[i] : (int)a.pup[i]) * a.P + pd;
          t0[r] = s_off[key];
          t1[r] = s_off[key + 1];
        }
        wold[r] = t1[r] > t0[r] ? wcol[i] : T(0);
      }
#pragma unroll
      for (int r = 0; r < kNdRows; ++r) {
        if (t1[r] == t0[r]) continue;
        const int64_t i = i0 + (int64_t)r * blockDim.x;
        T acc = T(0);
        for (int t = t0[r]; t < t1[r]; ++t)
          acc += s_amp[t] * vcol[i + s_du[t] + (int64_t)s_dd[t] * a.ld];
        const T add = acc * sc;
        wcol[i] = wold[r] + add;
        if (partial) dot += (double)(vcol[i] * sc) * (double)add;
      }
    }
  }
  if (partial) {
    const double s2 = block_sum(dot, red);
    if (threadIdx.x == 0) partial[blockIdx.x] = s2;
  }
}

int nd_blocks(const edx_sector* s) {
  return s->nd ? (int)std::min<int64_t>(s->ddw, kNdMaxBlocks) : 0;
}

// ---------------------------------------------------------------- planning
namespace {

constexpr size_t kSmallLdsBytes = 60 * 1024;
constexpr size_t kColLdsBytes = 150 * 1024;

size_t smem_header() { return kAmpTable * 8 + 64 * 8 + 16 * 8; }

}  // namespace

HvPlan hv_default_plan(const edx_sector* s, int vtype) {
  HvPlan p;
  const size_t sz = vbytes(vtype);
  const size_t bytes = (size_t)s->dim * sz;
  if (bytes + smem_header() <= kSmallLdsBytes) {
    p.mode = 0;
    p.col_blocks = 1;
    return p;
  }
  // One fused pass (spin-down neighbours gathered from global memory); it beat
  // the two-pass plan on every sector measured (Ns = 12..16, Norb = 1..3).
  // Columns per block: 2, or 3 for columns of 48 KB and more (the spin-up
  // table row is then reused over more columns), as far as LDS allows and
  // keeping a block per CU.
  const size_t colb = (size_t)s->dup * sz;
  const int ndt = nd_lds_terms(s);
  const size_t ndl = ndt > 0 ? 16 + nd_tab_lds(1 << s->model.norb, ndt, sz) : 0;
  int c = (int)std::max<size_t>(1, (kColLdsBytes - ndl) / colb);
  c = std::min(c, colb >= 48 * 1024 ? 3 : 2);
  while (c > 1 && (s->ddw + c - 1) / c < 256) --c;
  p.col_cols = c;
  p.col_threads = colb >= 48 * 1024 && c == 3 ? 1024 : 512;
  p.col_blocks = (int)((s->ddw + c - 1) / c);
  p.mode = 2;
  // XCD-contiguous groups inside windows all XCDs walk together (the L2 and
  // the MALL both see the shared spin-down neighbours): FP32 over the
  // pattern-sorted columns, FP64 (vectors twice the size) in listing order --
  // the faster of each on the Ns = 16 sector
  p.col_order = vtype == EDX_F32 ? 4 : 3;
  p.row_rows = (s->dup % 2 == 0) ? 128 : 64;
  p.row_cols = 8;
  return p;
}

edx_status hv_validate(const edx_sector* s, int vtype, HvPlan* p) {
  const size_t sz = vbytes(vtype);
  if (p->mode == 0) {
    if ((size_t)s->dim * sz + smem_header() > 160 * 1024) {
      set_error("hv plan: sector does not fit in LDS for mode 0");
      return EDX_E_UNSUPPORTED;
    }
    p->col_blocks = 1;
    return EDX_OK;
  }
  if (p->mode != 1 && p->mode != 2) {
    set_error("hv plan: mode must be 0, 1 or 2");
    return EDX_E_INVALID;
  }
  if (p->col_order < 0 || p->col_order > 4) {
    set_error("hv plan: col_order must be in [0, 4]");
    return EDX_E_INVALID;
  }
  if (p->col_cols < 1 || p->col_cols > kColMax ||
      (p->col_threads != 256 && p->col_threads != 512 && p->col_threads != 1024)) {
    set_error("hv plan: col_cols in [1, 4], col_threads in {256, 512, 1024}");
    return EDX_E_INVALID;
  }
  if (p->mode == 1 && ((p->row_rows != 16 && p->row_rows != 32 && p->row_rows != 64 &&
                        p->row_rows != 128) ||
                       p->row_cols < 1)) {
    set_error("hv plan: row_rows in {16, 32, 64, 128}, row_cols >= 1");
    return EDX_E_INVALID;
  }
  if (p->mode == 1 && p->row_rows == 128 && (s->dup & 1)) {
    set_error("hv plan: row_rows = 128 (two rows per lane) needs an even D_up");
    return EDX_E_UNSUPPORTED;
  }
  const size_t ndl = (nd_lds_terms(s) > 0 && p->mode == 2)
                         ? 16 + nd_tab_lds(1 << s->model.norb, nd_lds_terms(s), sz) : 0;
  if (smem_header() + (size_t)p->col_cols * s->dup * sz + 16 + ndl > 160 * 1024) {
    set_error("hv plan: columns do not fit in LDS");
    return EDX_E_UNSUPPORTED;
  }
  p->col_blocks = (int)((s->ddw + p->col_cols - 1) / p->col_cols);
  return EDX_OK;
}

HvPlan hv_plan(const edx_sector* s, int vtype) {
  const int k = vtype == EDX_F32 ? 1 : 0;
  if (!s->plan_set[k]) return hv_default_plan(s, vtype);
  return s->plan[k];
}

// partial sums of <v, Hv>: the last spin-separable pass's blocks, then the
// H_nd pass's
// partial sums of one electronic pass (one phonon slice)
static int hv_el_partial_blocks(const edx_sector* s, const HvPlan& p) {
  return p.col_blocks + (p.mode == 2 ? 0 : nd_blocks(s));
}

// workgroups of the phonon pass: groups of 8 columns per slice
static int ph_blocks(const edx_sector* s) { return (int)((s->ddw + 7) / 8) * s->dph; }

int hv_partial_blocks(const edx_sector* s, int vtype) {
  const HvPlan p = hv_plan(s, vtype);
  // the fused plan applies the phonon terms itself (per-slice term tables)
  return s->dph * hv_el_partial_blocks(s, p) + (s->dph > 1 && p.mode != 2 ? ph_blocks(s) : 0);
}

namespace {


template <typename T>
struct FusedOrder {
  int order;
  const int32_t* corder;
  NdTab<T> nd;   // nd.nt = 0: no spin exchange / pair hopping in this pass
  bool ph = false;   // phonon slice without H_nd: the direct phonon terms
  PhArgs<T> pa{};
};

template <typename T, int WUP, int WDW, int NC, bool ND, bool PH, bool BUF = false>
edx_status launch_fused_n(const HvArgs<T>& a, int nblk, int nthr, size_t lds, hipStream_t st,
                          const T* v, T* w, const double* vscale, double* partial,
                          FusedOrder<T> fo, const NdTab<T>& nd, uint32_t vbytes = 0) {
  const void* kern = (const void*)k_hv_fused<T, WUP, WDW, NC, ND, PH, BUF>;
  EDX_HIP(hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  hipLaunchKernelGGL((k_hv_fused<T, WUP, WDW, NC, ND, PH, BUF>), dim3(nblk), dim3(nthr), lds, st,
                     a, v, w, vscale, partial, fo.order, fo.corder, nd, fo.pa, vbytes);
  EDX_HIP(hipGetLastError());
  return EDX_OK;
}

template <typename T, int WUP, int WDW, int NC>
edx_status launch_fused_k(const HvArgs<T>& a, int nblk, int nthr, size_t lds, hipStream_t st,
                          const T* v, T* w, const double* vscale, double* partial,
                          FusedOrder<T> fo) {
  // buffer-load gathers when every byte offset into v (one phonon slice) fits
  // in 32 bits; the H_nd terms read outside it keep global loads.  The direct
  // phonon variant keeps global loads throughout (measured 2 % faster so, Ns=14
  // N_ph=4: 262-267 us against 270-271 us)
  const uint64_t vb = (uint64_t)a.ld * (uint64_t)a.ddw * sizeof(T);
  const bool buf = vb <= 0xFFFFFFFFull && a.hrow;
  if (fo.nd.nt > 0)
    return buf ? launch_fused_n<T, WUP, WDW, NC, true, false, true>(
                     a, nblk, nthr, lds, st, v, w, vscale, partial, fo, fo.nd, (uint32_t)vb)
               : launch_fused_n<T, WUP, WDW, NC, true, false>(a, nblk, nthr, lds, st, v, w,
                                                              vscale, partial, fo, fo.nd);
  if (fo.ph)
    return launch_fused_n<T, WUP, WDW, NC, false, true>(a, nblk, nthr, lds, st, v, w, vscale,
                                                        partial, fo, fo.nd);
  if (buf)
    return launch_fused_n<T, WUP, WDW, NC, false, false, true>(a, nblk, nthr, lds, st, v, w,
                                                               vscale, partial, fo, fo.nd,
                                                               (uint32_t)vb);
  return launch_fused_n<T, WUP, WDW, NC, false, false>(a, nblk, nthr, lds, st, v, w, vscale,
                                                       partial, fo, fo.nd);
}

template <typename T, int WUP, int WDW>
edx_status launch_fused_c(const HvArgs<T>& a, int ncol, int nblk, int nthr, size_t lds,
                          hipStream_t st, const T* v, T* w, const double* vscale,
                          double* partial, FusedOrder<T> fo) {
  switch (ncol) {
    case 1: return launch_fused_k<T, WUP, WDW, 1>(a, nblk, nthr, lds, st, v, w, vscale, partial, fo);
    case 2: return launch_fused_k<T, WUP, WDW, 2>(a, nblk, nthr, lds, st, v, w, vscale, partial, fo);
    case 3: return launch_fused_k<T, WUP, WDW, 3>(a, nblk, nthr, lds, st, v, w, vscale, partial, fo);
    default: return launch_fused_k<T, WUP, WDW, 4>(a, nblk, nthr, lds, st, v, w, vscale, partial, fo);
  }
}

template <typename T, int WUP>
edx_status launch_col_w(const HvArgs<T>& a, bool fused, int nblk, int nthr, size_t lds,
                        hipStream_t st, const T* v, T* w, const double* vscale, double* partial,
                        int ncol, FusedOrder<T> fo) {
  if (!fused) {
    EDX_HIP(hipFuncSetAttribute((const void*)k_hv_col<T, WUP>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    hipLaunchKernelGGL((k_hv_col<T, WUP>), dim3(nblk), dim3(nthr), lds, st, a, v, w, vscale,
                       partial, ncol, 1);
    EDX_HIP(hipGetLastError());
    return EDX_OK;
  }
  switch (a.sdw) {
    case 8: return launch_fused_c<T, WUP, 8>(a, ncol, nblk, nthr, lds, st, v, w, vscale, partial, fo);
    case 16: return launch_fused_c<T, WUP, 16>(a, ncol, nblk, nthr, lds, st, v, w, vscale, partial, fo);
    default: return launch_fused_c<T, WUP, 24>(a, ncol, nblk, nthr, lds, st, v, w, vscale, partial, fo);
  }
}

template <typename T, int R, int VEC>
edx_status launch_row_r(const HvArgs<T>& a, int64_t grid, hipStream_t st, const T* v, T* w,
                        const double* vscale, int64_t nchunk, int cpb, int64_t nwork) {
  switch (a.sdw) {
    case 8:
      hipLaunchKernelGGL((k_hv_row<T, R, VEC, 8>), dim3(grid), dim3(256), 0, st, a, v, w, vscale,
                         nchunk, cpb, nwork);
      break;
    case 16:
      hipLaunchKernelGGL((k_hv_row<T, R, VEC, 16>), dim3(grid), dim3(256), 0, st, a, v, w, vscale,
                         nchunk, cpb, nwork);
      break;
    default:
      hipLaunchKernelGGL((k_hv_row<T, R, VEC, 24>), dim3(grid), dim3(256), 0, st, a, v, w, vscale,
                         nchunk, cpb, nwork);
      break;
  }
  EDX_HIP(hipGetLastError());
  return EDX_OK;
}

template <typename T>
edx_status launch_t(const edx_sector* s, const T* v, T* w, int64_t ld, const double* vscale,
                    double* partial, hipStream_t st, const HvPlan& p, int slice) {
  HvArgs<T> a = make_args<T>(s, ld);
  const size_t hdr = smem_header();
  if (p.mode == 0) {
    const size_t lds = hdr + (size_t)s->dim * sizeof(T);
    if (lds > 160 * 1024) return EDX_E_UNSUPPORTED;
    EDX_HIP(hipFuncSetAttribute((const void*)k_hv_small<T>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    hipLaunchKernelGGL(k_hv_small<T>, dim3(1), dim3(1024), lds, st, a, v, w, vscale, partial);
    EDX_HIP(hipGetLastError());
    return EDX_OK;
  }
  if (p.col_cols > kColMax || p.col_cols < 1) return EDX_E_INVALID;
  // the fused pass also applies spin exchange / pair hopping from a staged table
  NdTab<T> nd{nullptr, nullptr, nullptr, nullptr, 1 << s->model.norb, 0};
  size_t ndl = 0;
  bool use_ph = false;
  PhArgs<T> pa{};
  if (p.mode == 2 && s->dph > 1 && slice >= 0 && !s->nd) {
    // phonon slice: W + w0 p, and the coupling to the neighbouring slices
    // read directly next to the gathers
    a.W = wph<T>(s) + (size_t)slice * 64;
    use_ph = true;
    pa.slice = ld * s->ddw;
    pa.sp = (T)std::sqrt((double)slice);
    pa.sp1 = (T)std::sqrt((double)(slice + 1));
    pa.g0 = (T)s->model.g[0];
    pa.g1 = (T)s->model.g[1];
    pa.g2 = (T)s->model.g[2];
    pa.lo = slice > 0;
    pa.hi = slice + 1 < s->dph;
  } else if (p.mode == 2 && s->dph > 1 && slice >= 0) {
    // phonon slice with H_nd: W + w0 p and the slice's merged term table
    const int P = 1 << s->model.norb;
    const int t0 = s->ph_start[slice], nt = s->ph_start[slice + 1] - t0;
    nd = NdTab<T>{s->ph_off + (size_t)slice * (P * P + 1), s->ph_du + t0, s->ph_dd + t0,
                  ph_amp<T>(s) + t0, P, nt};
    a.W = wph<T>(s) + (size_t)slice * 64;
    if (nt > 0) ndl = 16 + nd_tab_lds(nd.P, nd.nt, sizeof(T));
  } else if (s->nd && p.mode == 2) {
    nd = NdTab<T>{s->nd_off, s->nd_du, s->nd_dd, nd_amp<T>(s), 1 << s->model.norb, s->nd_nt};
    ndl = 16 + nd_tab_lds(nd.P, nd.nt, sizeof(T));
  }
  const size_t lds = hdr + (size_t)p.col_cols * s->dup * sizeof(T) + 16 + ndl;
  const int nthr = p.col_threads;
  if (lds > 160 * 1024) {
    set_error("hv: column does not fit in LDS (D_up too large)");
    return EDX_E_UNSUPPORTED;
  }
  const int nblk = (int)((s->ddw + p.col_cols - 1) / p.col_cols);
  if (p.mode == 1) {
    // spin-down rows first (writes w), then the column pass accumulates
    const int R = p.row_rows;
    const int64_t nslab = (s->dup + R - 1) / R;
    const int64_t nchunk = (s->ddw + p.row_cols - 1) / p.row_cols;
    const int64_t nwork = nslab * nchunk;
    const int64_t grid = ((nwork + 7) / 8) * 8;
    if (grid > 0x7FFFFFFF) return EDX_E_UNSUPPORTED;
    if (R == 16)
      EDX_TRY((launch_row_r<T, 16, 1>(a, grid, st, v, w, vscale, nchunk, p.row_cols, nwork)));
    else if (R == 32)
      EDX_TRY((launch_row_r<T, 32, 1>(a, grid, st, v, w, vscale, nchunk, p.row_cols, nwork)));
    else if (R == 64)
      EDX_TRY((launch_row_r<T, 64, 1>(a, grid, st, v, w, vscale, nchunk, p.row_cols, nwork)));
    else if (R == 128)
      EDX_TRY((launch_row_r<T, 64, 2>(a, grid, st, v, w, vscale, nchunk, p.row_cols, nwork)));
    else
      return EDX_E_INVALID;
  }
  const bool fused = p.mode == 2;
  // without the sorted column list, 2 falls back to 1 and 4 to 3
  FusedOrder<T> fo{s->corder ? p.col_order : (p.col_order == 4 ? 3 : std::min(p.col_order, 1)),
                   s->corder, nd};
  fo.ph = use_ph;
  fo.pa = pa;
  switch (a.sup) {
    case 8: return launch_col_w<T, 8>(a, fused, nblk, nthr, lds, st, v, w, vscale, partial, p.col_cols, fo);
    case 16: return launch_col_w<T, 16>(a, fused, nblk, nthr, lds, st, v, w, vscale, partial, p.col_cols, fo);
    default: return launch_col_w<T, 24>(a, fused, nblk, nthr, lds, st, v, w, vscale, partial, p.col_cols, fo);
  }
}

}  // namespace

namespace {

// Holstein terms (Sec. "Electron-phonon coupling", eq. HephBuild), added to the
// electronic product of every phonon slice p:
//   w_p += vs (w0 p v_p + G(i) (sqrt(p) v_{p-1} + sqrt(p+1) v_{p+1})),
//   G(i) = sum_a g_a (n_{a up} + n_{a dw}) from the two impurity patterns.
// Streams v three times (slices p-1, p, p+1) and w once each way; partial sums
// of <v, added terms> complete the Lanczos alpha of the electronic passes.
// Grid: x = groups of kPhCols columns of one slice, y = phonon slice; a block
// walks its columns row by row (coalesced, no index division).
constexpr int kPhCols = 8;

template <typename T>
__global__ __launch_bounds__(256) void k_hv_ph(const T* __restrict__ v, T* __restrict__ w,
                                               int64_t dup, int64_t ld, int64_t ddw, int dph,
                                               const uint8_t* __restrict__ pup,
                                               const uint8_t* __restrict__ pdw, int norb,
                                               double g0, double g1, double g2, double w0,
                                               const double* __restrict__ vscale,
                                               double* __restrict__ partial) {
  __shared__ double red[4];
  const double vs = vscale ? *vscale : 1.0;
  const int64_t slice = ld * ddw;
  const int p = blockIdx.y;
  const double wp = w0 * (double)p;
  const double sp = sqrt((double)p), sp1 = sqrt((double)(p + 1));
  const bool lo = p > 0, hi = p + 1 < dph;
  const int64_t j0 = (int64_t)blockIdx.x * kPhCols;
  const int64_t j1 = j0 + kPhCols < ddw ? j0 + kPhCols : ddw;
  double acc = 0.0;
  for (int64_t id = j0; id < j1; ++id) {
    const uint32_t pd = pdw[id];
    const int64_t base = (int64_t)p * slice + id * ld;
    for (int64_t iu = threadIdx.x; iu < dup; iu += blockDim.x) {
      const uint32_t pu = pup[iu];
      double gv = g0 * (double)((pu & 1u) + (pd & 1u));
      if (norb > 1) gv += g1 * (double)(((pu >> 1) & 1u) + ((pd >> 1) & 1u));
      if (norb > 2) gv += g2 * (double)(((pu >> 2) & 1u) + ((pd >> 2) & 1u));
      const int64_t idx = base + iu;
      const double x = (double)v[idx];
      double res = wp * x;
      if (lo) res += gv * sp * (double)v[idx - slice];
      if (hi) res += gv * sp1 * (double)v[idx + slice];
      res *= vs;
      w[idx] = (T)((double)w[idx] + res);
      acc += x * vs * res;
    }
  }
  const double sum = block_sum(acc, red);
  if (partial && threadIdx.x == 0) partial[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] = sum;
}

// the electronic product on one slice (column stride ld, D_dw columns)
edx_status hv_launch_el(const edx_sector* s, int vtype, const void* v, void* w, int64_t ld,
                        const double* vscale, double* partial, hipStream_t st,
                        const HvPlan* plan, int slice) {
  HvPlan p = plan ? *plan : hv_plan(s, vtype);
  if (ld < s->dup) {
    set_error("hv: leading dimension below D_up");
    return EDX_E_INVALID;
  }
  // two rows per lane uses 8/16-byte loads: only for 16-byte aligned vectors
  // whose columns all start on an even element
  if (p.mode == 1 && p.row_rows == 128 &&
      (((reinterpret_cast<uintptr_t>(v) | reinterpret_cast<uintptr_t>(w)) & 15u) || (ld & 1)))
    p.row_rows = 64;
  if (vtype == EDX_F64)
    EDX_TRY(launch_t<double>(s, static_cast<const double*>(v), static_cast<double*>(w), ld,
                             vscale, partial, st, p, slice));
  else
    EDX_TRY(launch_t<float>(s, static_cast<const float*>(v), static_cast<float*>(w), ld, vscale,
                            partial, st, p, slice));
  if (!s->nd || p.mode == 2) return EDX_OK;
  const int nb = nd_blocks(s);
  double* pnd = partial ? partial + p.col_blocks : nullptr;
  const int P = 1 << s->model.norb;
  const size_t patlds = s->dup <= kNdPatLds ? (size_t)s->dup : 0;
  if (vtype == EDX_F64) {
    const NdArgs<double> na{s->dup, s->ddw, ld, s->up.pat, s->dw.pat, s->nd_off, s->nd_du,
                            s->nd_dd, s->nd_amp64, P};
    hipLaunchKernelGGL(k_hv_nd<double>, dim3(nb), dim3(256), patlds, st, na,
                       static_cast<const double*>(v), static_cast<double*>(w), vscale, pnd);
  } else {
    const NdArgs<float> na{s->dup, s->ddw, ld, s->up.pat, s->dw.pat, s->nd_off, s->nd_du,
                           s->nd_dd, s->nd_amp32, P};
    hipLaunchKernelGGL(k_hv_nd<float>, dim3(nb), dim3(256), patlds, st, na,
                       static_cast<const float*>(v), static_cast<float*>(w), vscale, pnd);
  }
  EDX_HIP(hipGetLastError());
  return EDX_OK;
}

}  // namespace

edx_status hv_launch(const edx_sector* s, int vtype, const void* v, void* w, int64_t ld,
                     const double* vscale, double* partial, hipStream_t st,
                     const HvPlan* plan) {
  if (s->dph <= 1) return hv_launch_el(s, vtype, v, w, ld, vscale, partial, st, plan, -1);
  if (ld < s->dup) {
    set_error("hv: leading dimension below D_up");
    return EDX_E_INVALID;
  }
  const HvPlan p = plan ? *plan : hv_plan(s, vtype);
  const int eb = hv_el_partial_blocks(s, p);
  const size_t sb = (size_t)(ld * s->ddw) * vbytes(vtype);
  // fused plan: each slice's pass applies its phonon terms (term table); the
  // other plans add them in a separate pass
  const bool fused = p.mode == 2;
  for (int q = 0; q < s->dph; ++q)
    EDX_TRY(hv_launch_el(s, vtype, static_cast<const char*>(v) + q * sb,
                         static_cast<char*>(w) + q * sb, ld, vscale,
                         partial ? partial + (size_t)q * eb : nullptr, st, &p, fused ? q : -1));
  if (fused) return EDX_OK;
  double* pph = partial ? partial + (size_t)s->dph * eb : nullptr;
  const Model& m = s->model;
  const dim3 grid((unsigned)((s->ddw + kPhCols - 1) / kPhCols), (unsigned)s->dph);
  if (vtype == EDX_F64)
    hipLaunchKernelGGL(k_hv_ph<double>, grid, dim3(256), 0, st,
                       static_cast<const double*>(v), static_cast<double*>(w), s->dup, ld,
                       s->ddw, s->dph, s->up.pat, s->dw.pat, m.norb, m.g[0], m.g[1], m.g[2],
                       m.w0, vscale, pph);
  else
    hipLaunchKernelGGL(k_hv_ph<float>, grid, dim3(256), 0, st,
                       static_cast<const float*>(v), static_cast<float*>(w), s->dup, ld,
                       s->ddw, s->dph, s->up.pat, s->dw.pat, m.norb, m.g[0], m.g[1], m.g[2],
                       m.w0, vscale, pph);
  EDX_HIP(hipGetLastError());
  return EDX_OK;
}

// Column pass of the distributed pieces on a column block (edx_hv_block):
// w = (H_d + H_up) V over NC columns per workgroup, overwriting.  The fused
// pass's row machinery without the spin-down gathers: interleaved LDS columns
// at offset 0, compact hop rows, buffer loads and streaming buffer stores
// (every byte offset into the block below 2^32, D < 2^16).
template <typename T, int WUP, int NC>
__global__ __launch_bounds__(1024) void k_hv_colx(HvArgs<T> a, const T* __restrict__ v,
                                                  T* __restrict__ w, uint32_t vbytes) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* vs = reinterpret_cast<T*>(smem_raw);
  T* amp = reinterpret_cast<T*>(smem_raw + al16((size_t)NC * a.dup * sizeof(T)));
  T* Wt = amp + kAmpTable;
  const uint32_t dup = (uint32_t)a.dup;
  const int64_t ld = a.ld;
  const int64_t j0 = (int64_t)blockIdx.x * NC;
  const int nc = (int)std::min<int64_t>(NC, a.ddw - j0);
  constexpr int HW = 3 * WUP / 4;
  const __amdgpu_buffer_rsrc_t vres =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<T*>(v), 0, (int)vbytes, 0x00020000);
  const __amdgpu_buffer_rsrc_t wres = __builtin_amdgcn_make_buffer_rsrc(w, 0, (int)vbytes,
                                                                        0x00020000);
  const __amdgpu_buffer_rsrc_t hres = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<uint8_t*>(a.hrow), 0, (int)(dup * HW * 4), 0x00020000);
  const __amdgpu_buffer_rsrc_t eres = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<T*>(a.eup), 0, (int)(dup * sizeof(T)), 0x00020000);
  const __amdgpu_buffer_rsrc_t pres = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<uint8_t*>(a.pup), 0, (int)dup, 0x00020000);
  uint32_t coff[NC];
  T ed[NC];
  int pd[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const int64_t j = std::min<int64_t>(j0 + c, a.ddw - 1);   // clamped copies past the end
    coff[c] = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)j * ld * sizeof(T)));
    ed[c] = a.edw[j];
    pd[c] = a.pdw[j];
  }
  constexpr int SU = std::max(1, (sizeof(T) == 4 ? 40 : 20) / NC);
  StageBuf<T, NC, SU> sb;
  stage_issue_buf(sb, vres, coff, nc, dup, threadIdx.x);
  for (int i = threadIdx.x; i < kAmpTable; i += blockDim.x) amp[i] = a.amp[i];
  for (int i = threadIdx.x; i < 64; i += blockDim.x) Wt[i] = a.W[i];
  stage_put(vs, sb, nc, (int64_t)dup, (int64_t)threadIdx.x, T(1));
  for (uint32_t r0 = threadIdx.x + SU * blockDim.x; r0 < dup; r0 += SU * blockDim.x) {
    stage_issue_buf(sb, vres, coff, nc, dup, r0);
    stage_put(vs, sb, nc, (int64_t)dup, (int64_t)r0, T(1));
  }
  __syncthreads();
  for (uint32_t iu = threadIdx.x; iu < dup; iu += blockDim.x) {
    const uint32_t voff = iu * (uint32_t)sizeof(T);
    uint32_t r[HW];
#pragma unroll
    for (int q = 0; q < HW / 2; ++q) {
      typedef unsigned int u2 __attribute__((ext_vector_type(2)));
      const u2 x = __builtin_amdgcn_raw_buffer_load_b64(hres, (int)(iu * HW * 4 + q * 8), 0, 0);
      r[2 * q] = x.x;
      r[2 * q + 1] = x.y;
    }
    const T eu = buf_load<T>(eres, voff, 0);
    const int pu = (int)__builtin_amdgcn_raw_buffer_load_b8(pres, (int)iu, 0, 0) * 8;
    T acc[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) acc[c] = T(0);
#pragma unroll
    for (int k = 0; k < WUP; ++k) {
      const uint32_t col = (r[k >> 1] >> (16 * (k & 1))) & 0xFFFFu;
      const uint32_t ai = (r[WUP / 2 + (k >> 2)] >> (8 * (k & 3))) & 0xFFu;
      const T am = amp[ai];
      const T* src = vs + __umul24(col, (uint32_t)NC);
#pragma unroll
      for (int c = 0; c < NC; ++c) acc[c] += am * src[c];
    }
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      if (c >= nc) break;
      const T x = vs[iu * (uint32_t)NC + c];
      buf_store_nt<T>(wres, voff, coff[c], acc[c] + (eu + ed[c] + Wt[pu + pd[c]]) * x);
    }
  }
  // padding rows of the output are defined as zero
  for (int64_t i = (int64_t)dup + threadIdx.x; i < ld; i += blockDim.x)
#pragma unroll
    for (int c = 0; c < NC; ++c)
      if (c < nc) w[i + (j0 + c) * ld] = T(0);
}

// ---------------------------------------------------------------- distributed pieces
// The per-GPU work of the column-distributed product (Sec. 3.2, two transposes
// per product), run on one GPU: part 0 is the local pass on a column block of V
// (spin-up hops inside the columns plus H_d), part 1 the pass on a column block
// of the transposed vector V^T (D_dw x D_up, spin-down hops inside its columns,
// no diagonal).  Both are the column pass of the two-pass plan on a shifted
// view: for part 1 the roles of the two spins swap and the diagonal tables are
// replaced by zeros.  Output columns are overwritten.
namespace {

template <typename T>
edx_status block_t(const edx_sector* s, int part, const T* v, T* w, int64_t ld, int64_t c0,
                   int64_t c1, hipStream_t st) {
  HvArgs<T> a = make_args<T>(s, ld);
  const T* zt = reinterpret_cast<const T*>(s->zeros);
  if (part == 0) {
    a.ddw = c1 - c0;
    a.edw += c0;
    a.pdw += c0;
  } else {
    a.dup = s->ddw;
    a.ddw = c1 - c0;
    a.hup = s->dw.hop;
    a.sup = s->dw.wpad;
    a.hdw = s->up.hop;
    a.sdw = s->up.wpad;
    a.eup = zt;
    a.edw = zt;
    a.pup = s->dw.pat;
    a.pdw = s->up.pat + c0;
    a.W = zt;
  }
  const int64_t len = a.dup;
  // several columns per workgroup only while that still leaves >= 4
  // workgroups per CU (narrow blocks of a p-way split)
  int C = 1;
  for (int c = 3; c >= 2; --c)
    if (smem_header() + (size_t)c * len * sizeof(T) <= 150 * 1024 && a.ddw / c >= 1024) {
      C = c;
      break;
    }
  const size_t lds = smem_header() + (size_t)C * len * sizeof(T);
  if (lds > 160 * 1024) {
    set_error("hv_block: column does not fit in LDS");
    return EDX_E_UNSUPPORTED;
  }
  const int nthr = C == 3 ? 1024 : 512;
  const int nblk = (int)((a.ddw + C - 1) / C);
  const T* vb = v + c0 * ld;
  T* wb = w + c0 * ld;
  // compact-row pass when the block's byte offsets fit in 32 bits
  const uint8_t* hr = part == 0 ? s->hrow : s->hrow_dw;
  const uint64_t bytes = (uint64_t)a.ddw * (uint64_t)ld * sizeof(T);
  if (hr && bytes <= 0xFFFFFFFFull) {
    a.hrow = hr;
    const size_t ldsx = smem_header() + 16 + (size_t)C * len * sizeof(T);
    auto gox = [&](auto kern) -> edx_status {
      EDX_HIP(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)ldsx));
      hipLaunchKernelGGL(kern, dim3(nblk), dim3(nthr), ldsx, st, a, vb, wb, (uint32_t)bytes);
      EDX_HIP(hipGetLastError());
      return EDX_OK;
    };
    auto byc = [&](auto w8) -> edx_status {
      constexpr int W = decltype(w8)::value;
      switch (C) {
        case 1: return gox(k_hv_colx<T, W, 1>);
        case 2: return gox(k_hv_colx<T, W, 2>);
        default: return gox(k_hv_colx<T, W, 3>);
      }
    };
    switch (a.sup) {
      case 8: return byc(std::integral_constant<int, 8>{});
      case 16: return byc(std::integral_constant<int, 16>{});
      default: return byc(std::integral_constant<int, 24>{});
    }
  }
  auto go = [&](auto kern) -> edx_status {
    EDX_HIP(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)lds));
    hipLaunchKernelGGL(kern, dim3(nblk), dim3(nthr), lds, st, a, vb, wb, nullptr, nullptr, C, 0);
    EDX_HIP(hipGetLastError());
    return EDX_OK;
  };
  switch (a.sup) {
    case 8: return go(k_hv_col<T, 8>);
    case 16: return go(k_hv_col<T, 16>);
    default: return go(k_hv_col<T, 24>);
  }
}

// dst (cols x rows, stride ldd) = src^T (+ dst if add); src is rows x cols with
// stride lds.  64 x 64 tiles through LDS (padded rows: no bank conflicts), so
// both the reads and the writes are coalesced.
template <typename T>
__global__ __launch_bounds__(256) void k_transpose_t(const T* __restrict__ src, int64_t rows,
                                                     int64_t cols, int64_t lds,
                                                     T* __restrict__ dst, int64_t ldd, int add,
                                                     int64_t tiles_r) {
  __shared__ T tile[64][65];
  const int64_t tr = blockIdx.x % tiles_r;
  const int64_t tc = blockIdx.x / tiles_r;
  const int tx = threadIdx.x & 63;
  const int ty = threadIdx.x >> 6;   // 0..3
  const int64_t r0 = tr * 64, c0 = tc * 64;
  for (int k = ty; k < 64; k += 4) {
    const int64_t r = r0 + tx, c = c0 + k;
    if (r < rows && c < cols) tile[k][tx] = src[r + c * lds];
  }
  __syncthreads();
  for (int k = ty; k < 64; k += 4) {
    const int64_t c = c0 + tx, r = r0 + k;   // dst element (c, r)
    if (r < rows && c < cols) {
      const T x = tile[tx][k];
      T* d = dst + c + r * ldd;
      *d = add ? (T)(*d + x) : x;
    }
  }
}

}  // namespace

edx_status hv_block_launch(const edx_sector* s, int vtype, int part, const void* v, void* w,
                           int64_t ld, int64_t c0, int64_t c1, hipStream_t st) {
  if (vtype == EDX_F64)
    return block_t<double>(s, part, static_cast<const double*>(v), static_cast<double*>(w), ld,
                           c0, c1, st);
  return block_t<float>(s, part, static_cast<const float*>(v), static_cast<float*>(w), ld, c0,
                        c1, st);
}

edx_status k_transpose(int vtype, const void* src, int64_t rows, int64_t cols, int64_t lds,
                       void* dst, int64_t ldd, int add, hipStream_t st) {
  const int64_t tr = (rows + 63) / 64, tcn = (cols + 63) / 64;
  const int64_t nb = tr * tcn;
  if (nb > 0x7FFFFFFF) {
    set_error("transpose: too many tiles");
    return EDX_E_UNSUPPORTED;
  }
  if (nb == 0) return EDX_OK;
  if (vtype == EDX_F64)
    hipLaunchKernelGGL(k_transpose_t<double>, dim3((unsigned)nb), dim3(256), 0, st,
                       static_cast<const double*>(src), rows, cols, lds,
                       static_cast<double*>(dst), ldd, add, tr);
  else
    hipLaunchKernelGGL(k_transpose_t<float>, dim3((unsigned)nb), dim3(256), 0, st,
                       static_cast<const float*>(src), rows, cols, lds, static_cast<float*>(dst),
                       ldd, add, tr);
  EDX_HIP(hipGetLastError());
  return EDX_OK;
}

edx_status hv_autotune(edx_sector* s, int vtype, const void* v, void* w, int64_t ld, int reps,
                       hipStream_t st, HvPlan* best, double* best_us) {
  std::vector<HvPlan> cands;
  auto add = [&](HvPlan p) {
    if (hv_validate(s, vtype, &p) == EDX_OK) cands.push_back(p);
  };
  {
    HvPlan p;
    p.mode = 0;
    add(p);
  }
  for (int cc : {1, 2, 3, 4})
    for (int th : {256, 512, 1024}) {
      HvPlan p;
      p.mode = 2;
      p.col_cols = cc;
      p.col_threads = th;
      for (int co : {0, 1, 2, 3, 4}) {
        HvPlan r = p;
        r.col_order = co;
        add(r);
      }
      for (int rr : {32, 64, 128})
        for (int rc : {8, 32}) {
          HvPlan q = p;
          q.mode = 1;
          q.row_rows = rr;
          q.row_cols = rc;
          add(q);
        }
    }
  set_error("");
  if (cands.empty()) {
    set_error("autotune: no plan fits this sector");
    return EDX_E_UNSUPPORTED;
  }
  hipEvent_t e0, e1;
  EDX_HIP(hipEventCreate(&e0));
  EDX_HIP(hipEventCreate(&e1));
  double best_t = 1e300;
  HvPlan bp = cands[0];
  for (const HvPlan& p : cands) {
    EDX_TRY(hv_launch(s, vtype, v, w, ld, nullptr, nullptr, st, &p));   // warm-up
    EDX_HIP(hipEventRecord(e0, st));
    for (int r = 0; r < reps; ++r) EDX_TRY(hv_launch(s, vtype, v, w, ld, nullptr, nullptr, st, &p));
    EDX_HIP(hipEventRecord(e1, st));
    EDX_HIP(hipEventSynchronize(e1));
    float ms = 0.f;
    EDX_HIP(hipEventElapsedTime(&ms, e0, e1));
    const double us = 1000.0 * ms / std::max(1, reps);
    if (us < best_t) {
      best_t = us;
      bp = p;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  const int k = vtype == EDX_F32 ? 1 : 0;
  s->plan[k] = bp;
  s->plan_set[k] = true;
  if (best) *best = bp;
  if (best_us) *best_us = best_t;
  return EDX_OK;
}

}  // namespace edx
