// Storage-free H.v for one sector (Sec. 3 "Matrix-vector product", eq. Hbuild).
//
// With v viewed as the D_up x D_dw column-major matrix V of eq. Vmatrix,
//   W = H_d o V + H_up V + V H_dw^T.
// The spin-up hops stay inside a column (contiguous), the spin-down hops stay
// inside a row (stride D_up).  The paper makes the row access local with an MPI
// transpose (Sec. 3.2).  One GPU holds the whole vector, so instead:
//
//  * k_hv_col  -- one block per group of consecutive columns; the columns are
//                 staged in LDS, so the spin-up gathers hit LDS.  Adds H_d.
//                 Fused variant: also gathers the spin-down neighbours of each
//                 element straight from global memory (whole neighbour
//                 columns, coalesced; pays off when the vector is cache
//                 resident).
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
#include <algorithm>
#include <vector>

#include "common.cuh"
#include "edx_internal.h"

namespace edx {

template <typename T>
struct HvArgs {
  int64_t dup, ddw;
  const uint32_t* __restrict__ hup;   // row-major, stride sup
  const uint32_t* __restrict__ hdw;   // row-major, stride sdw
  int sup, sdw;                       // padded row lengths (8, 16 or 24)
  const T* __restrict__ eup;
  const T* __restrict__ edw;
  const uint8_t* __restrict__ pup;
  const uint8_t* __restrict__ pdw;
  const T* __restrict__ amp;   // [256]
  const T* __restrict__ W;     // [64]
};

template <typename T>
HvArgs<T> make_args(const edx_sector* s);

template <>
HvArgs<double> make_args<double>(const edx_sector* s) {
  return HvArgs<double>{s->dup, s->ddw, s->up.hop, s->dw.hop, s->up.wpad, s->dw.wpad,
                        s->up.e64, s->dw.e64, s->up.pat, s->dw.pat, s->amp64, s->w64};
}
template <>
HvArgs<float> make_args<float>(const edx_sector* s) {
  return HvArgs<float>{s->dup, s->ddw, s->up.hop, s->dw.hop, s->up.wpad, s->dw.wpad,
                       s->up.e32, s->dw.e32, s->up.pat, s->dw.pat, s->amp32, s->w32};
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
  for (int64_t i = threadIdx.x; i < D; i += blockDim.x) vs[i] = v[i] * sc;
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
    w[idx] = acc;
    dot += (double)x * (double)acc;
  }
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

template <typename T>
__device__ __forceinline__ void stage(T* __restrict__ vs, const T* __restrict__ src, int64_t n,
                                      T sc) {
  const int bd = blockDim.x;
  int64_t i = threadIdx.x;
  for (; i + 7 * bd < n; i += 8 * bd) {
    T x[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) x[u] = src[i + u * bd];
#pragma unroll
    for (int u = 0; u < 8; ++u) vs[i + u * bd] = x[u] * sc;
  }
  for (; i < n; i += bd) vs[i] = src[i] * sc;
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

template <typename T, int WUP, int WDW, bool FUSE_DW, bool ACCUM>
__global__ __launch_bounds__(1024) void k_hv_col(HvArgs<T> a, const T* __restrict__ v,
                                                 T* __restrict__ w,
                                                 const double* __restrict__ vscale,
                                                 double* __restrict__ partial, int ncol) {
  constexpr int RPT = FUSE_DW ? 1 : 2;   // rows per thread per iteration
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
  stage(vs, v + j0 * dup, (int64_t)nc * dup, sc);
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
      if (ACCUM) {
#pragma unroll
        for (int c = 0; c < kColMax; ++c)
          wold[r][c] = c < nc ? w[rows[r] + jc[c] * dup] : T(0);
      }
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
        T res = acc[c] + (eu[r] + ed[c] + Wt[pu[r] + pd[c]]) * x;
        if (FUSE_DW) {
          uint32_t f[WDW];
#pragma unroll
          for (int k = 0; k < WDW; ++k) f[k] = a.hdw[j * WDW + k];
          T g[WDW];
#pragma unroll
          for (int k = 0; k < WDW; ++k) g[k] = v[iu + (int64_t)(f[k] & kColMask) * dup];
          T s2 = T(0);
#pragma unroll
          for (int k = 0; k < WDW; ++k) s2 += amp[f[k] >> kAmpShift] * g[k];
          res += s2 * sc;
        }
        if (ACCUM) res += wold[r][c];
        w[iu + j * dup] = res;
        dot += (double)x * (double)res;
      }
    }
  }
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
      g1[k] = *reinterpret_cast<const V*>(v + iuc + (int64_t)(e1[k] & kColMask) * a.dup);
      g2[k] = *reinterpret_cast<const V*>(v + iuc + (int64_t)(e2[k] & kColMask) * a.dup);
    }
    V s1 = V(0), s2 = V(0);
#pragma unroll
    for (int k = 0; k < WDW; ++k) {
      s1 += (amp[e1[k] >> kAmpShift] * sc) * g1[k];
      s2 += (amp[e2[k] >> kAmpShift] * sc) * g2[k];
    }
    // streaming stores: keep L2 for the slab being gathered
    if (ok) {
      __builtin_nontemporal_store(s1, reinterpret_cast<V*>(w + iu + j * a.dup));
      if (has2) __builtin_nontemporal_store(s2, reinterpret_cast<V*>(w + iu + j2 * a.dup));
    }
  }
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
  // columns per block: fill LDS up to kColLdsBytes, but keep >= ~1024 blocks
  int c = (int)std::max<size_t>(1, kColLdsBytes / ((size_t)s->dup * sz));
  c = std::min(c, kColMax);
  while (c > 1 && (s->ddw + c - 1) / c < 1024) --c;
  p.col_cols = c;
  p.col_threads = 512;
  p.col_blocks = (int)((s->ddw + c - 1) / c);
  // the fused single pass reads whole neighbour columns from global memory; it
  // is the right choice while the vector is cache resident
  p.mode = bytes <= (size_t)32 * 1024 * 1024 ? 2 : 1;
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
  if (smem_header() + (size_t)p->col_cols * s->dup * sz > 160 * 1024) {
    set_error("hv plan: columns do not fit in LDS");
    return EDX_E_UNSUPPORTED;
  }
  p->col_blocks = (int)((s->ddw + p->col_cols - 1) / p->col_cols);
  return EDX_OK;
}

HvPlan hv_plan(const edx_sector* s, int vtype) {
  const int k = vtype == EDX_F32 ? 1 : 0;
  if (!s->plan_set[k]) return hv_default_plan(s, vtype);
  HvPlan p;
  p.mode = s->plan_v[k][0];
  p.col_cols = s->plan_v[k][1];
  p.col_threads = s->plan_v[k][2];
  p.row_rows = s->plan_v[k][3];
  p.row_cols = s->plan_v[k][4];
  p.col_blocks = s->plan_v[k][5];
  return p;
}

int hv_partial_blocks(const edx_sector* s, int vtype) { return hv_plan(s, vtype).col_blocks; }

namespace {


template <typename T, int WUP, int WDW>
edx_status launch_col(const HvArgs<T>& a, bool fused, int nblk, int nthr, size_t lds,
                      hipStream_t st, const T* v, T* w, const double* vscale, double* partial,
                      int ncol) {
  const void* kern = fused ? (const void*)k_hv_col<T, WUP, WDW, true, false>
                           : (const void*)k_hv_col<T, WUP, WDW, false, true>;
  EDX_HIP(hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  if (fused)
    hipLaunchKernelGGL((k_hv_col<T, WUP, WDW, true, false>), dim3(nblk), dim3(nthr), lds, st, a,
                       v, w, vscale, partial, ncol);
  else
    hipLaunchKernelGGL((k_hv_col<T, WUP, WDW, false, true>), dim3(nblk), dim3(nthr), lds, st, a,
                       v, w, vscale, partial, ncol);
  EDX_HIP(hipGetLastError());
  return EDX_OK;
}

template <typename T, int WUP>
edx_status launch_col_w(const HvArgs<T>& a, bool fused, int nblk, int nthr, size_t lds,
                        hipStream_t st, const T* v, T* w, const double* vscale, double* partial,
                        int ncol) {
  if (!fused)   // the spin-down width does not enter the accumulate variant
    return launch_col<T, WUP, 8>(a, false, nblk, nthr, lds, st, v, w, vscale, partial, ncol);
  switch (a.sdw) {
    case 8: return launch_col<T, WUP, 8>(a, true, nblk, nthr, lds, st, v, w, vscale, partial, ncol);
    case 16: return launch_col<T, WUP, 16>(a, true, nblk, nthr, lds, st, v, w, vscale, partial, ncol);
    default: return launch_col<T, WUP, 24>(a, true, nblk, nthr, lds, st, v, w, vscale, partial, ncol);
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
edx_status launch_t(const edx_sector* s, const T* v, T* w, const double* vscale,
                    double* partial, hipStream_t st, const HvPlan& p) {
  const HvArgs<T> a = make_args<T>(s);
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
  const size_t lds = hdr + (size_t)p.col_cols * s->dup * sizeof(T);
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
  switch (a.sup) {
    case 8: return launch_col_w<T, 8>(a, fused, nblk, nthr, lds, st, v, w, vscale, partial, p.col_cols);
    case 16: return launch_col_w<T, 16>(a, fused, nblk, nthr, lds, st, v, w, vscale, partial, p.col_cols);
    default: return launch_col_w<T, 24>(a, fused, nblk, nthr, lds, st, v, w, vscale, partial, p.col_cols);
  }
}

}  // namespace

edx_status hv_launch(const edx_sector* s, int vtype, const void* v, void* w,
                     const double* vscale, double* partial, hipStream_t st,
                     const HvPlan* plan) {
  HvPlan p = plan ? *plan : hv_plan(s, vtype);
  // two rows per lane uses 8/16-byte loads: only for 16-byte aligned vectors
  if (p.mode == 1 && p.row_rows == 128 &&
      ((reinterpret_cast<uintptr_t>(v) | reinterpret_cast<uintptr_t>(w)) & 15u))
    p.row_rows = 64;
  if (vtype == EDX_F64)
    return launch_t<double>(s, static_cast<const double*>(v), static_cast<double*>(w), vscale,
                            partial, st, p);
  return launch_t<float>(s, static_cast<const float*>(v), static_cast<float*>(w), vscale,
                         partial, st, p);
}

edx_status hv_autotune(edx_sector* s, int vtype, const void* v, void* w, int reps,
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
      add(p);
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
    EDX_TRY(hv_launch(s, vtype, v, w, nullptr, nullptr, st, &p));   // warm-up
    EDX_HIP(hipEventRecord(e0, st));
    for (int r = 0; r < reps; ++r) EDX_TRY(hv_launch(s, vtype, v, w, nullptr, nullptr, st, &p));
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
  s->plan_v[k][0] = bp.mode;
  s->plan_v[k][1] = bp.col_cols;
  s->plan_v[k][2] = bp.col_threads;
  s->plan_v[k][3] = bp.row_rows;
  s->plan_v[k][4] = bp.row_cols;
  s->plan_v[k][5] = bp.col_blocks;
  s->plan_set[k] = true;
  if (best) *best = bp;
  if (best_us) *best_us = best_t;
  return EDX_OK;
}

}  // namespace edx
