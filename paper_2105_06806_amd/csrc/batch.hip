// Batched ground states of many sectors.
//
// Jobs whose dimension reaches a threshold (wide_min) fill the GPU by
// themselves: they run first, one after another, through the whole-GPU
// kernels of the plain path (lanczos.hip).  All other jobs share one
// persistent launch: the grid is one workgroup per CU, launched cooperatively
// so that every workgroup is resident.  Workgroups are grouped into lanes of L workgroups
// that sit on one XCD (workgroup b runs on XCD b % 8), so a lane shares one L2.
// A lane pulls the next job from a device queue (jobs sorted by decreasing
// dimension), runs the whole Lanczos recurrence of Sec. 6 "Diagonalization" for
// it, writes E0 and takes the next job; lanes synchronise internally with a
// counter barrier (bounded spin: a stuck lane reports an error instead of
// hanging).  Inside a lane a step is the same sequence as the plain path:
//   row pass (spin-down hops, slabs of 64 rows, the slab stays in the XCD's L2)
//   -> column pass (LDS-staged columns: diagonal + spin-up hops, <v, Hv>)
//   -> three-term update with |w|^2 -> beta, scale.
// The stop rule |E_j - E_{j-1}| <= tol max(1, |E_j|), breakdown or niter is
// evaluated on the device every `check_every` steps: one wave finds the lowest
// eigenvalue of T_j by multisection (64 Sturm counts per round), redundantly and
// identically in every workgroup of the lane, so no broadcast is needed.
// Dot products accumulate in FP64 with a fixed reduction order.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <string>
#include <thread>
#include <vector>

#include "common.h"
#include "edx_internal.h"

namespace edx {

struct BatchJob {
  const uint32_t* hup;
  const uint32_t* hdw;
  const void* eup;
  const void* edw;
  const uint8_t* pup;
  const uint8_t* pdw;
  const void* amp;
  const void* W;
  int64_t dup, ddw;
  int sup, sdw;
  int ccols;        // columns per column-pass item
  int rcols;        // columns per row-pass item
  int pad0, pad1;
};

struct BatchOut {
  double e0;
  double beta_last;
  int iters;
  int status;       // 0 ok, 4 no convergence, 3 device (barrier timeout)
  int breakdown;
  int pad;
};

namespace {

constexpr int kThreads = 1024;
constexpr int kWaves = kThreads / 64;
constexpr long long kSpinLimit = 1ll << 26;
constexpr int kColMaxB = 4;   // columns per column-pass item held in registers
constexpr int kMaxBatchIter = 2048;   // niter bound of the batch call
// Whole-GPU jobs run on this many streams at once (one host thread each), so
// that one job's kernels fill the gaps while another's host checks its stop
// rule.
constexpr int kWideStreams = 3;
constexpr int kMultiDefault = 8;        // bath sets per multi-set group (tiles.multi_k = 0)
// Shapes the multi-set pass serves: up to 2^21 states, at most 4 FP64 sets.
// Measured per vector against the single-set fused pass: half-filled Ns=12
// (D = 853,776) 5.3 vs 10.1 us (FP32, 4 or 8 sets), 9.2-9.8 vs 11.3 us (FP64,
// 2 or 4 sets; 8 sets 12.3 us); Ns=14 (D = 11.8M) 58-68 vs 48 us (FP32) --
// there one column of k sets is k times the footprint in L2, so the misses
// per vector do not fall while the grid is already full.
constexpr int64_t kMultiMaxDim = int64_t(1) << 21;
constexpr int kMultiMaxF64 = 4;

__device__ __forceinline__ uint64_t splitmix64(uint64_t seed, uint64_t k) {
  uint64_t z = seed + (k + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Barrier over the L workgroups of a lane.  `gen` counts the barriers passed
// by this workgroup; all workgroups of a lane pass the same sequence.
__device__ bool lane_barrier(unsigned* ctr, unsigned& gen, int L, int* err) {
  __syncthreads();
  __shared__ int fail;
  if (threadIdx.x == 0) {
    fail = 0;
    __threadfence();
    atomicAdd(ctr, 1u);
    const unsigned target = (gen + 1) * (unsigned)L;
    long long spins = 0;
    while (__hip_atomic_load(ctr, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < target) {
      if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0 ||
          ++spins > kSpinLimit) {
        atomicExch(err, 1);
        fail = 1;
        break;
      }
      __builtin_amdgcn_s_sleep(2);
    }
    __threadfence();
  }
  __syncthreads();
  ++gen;
  return fail == 0;
}

// number of eigenvalues of T_m below x (Sturm sequence)
__device__ int sturm(const double* a, const double* b, int m, double x) {
  int cnt = 0;
  double q = a[0] - x;
  cnt += q < 0.0;
  for (int i = 1; i < m; ++i) {
    if (fabs(q) < 1e-300) q = -1e-300;
    q = a[i] - x - b[i] * b[i] / q;   // b[i] couples i-1 and i
    cnt += q < 0.0;
  }
  return cnt;
}

// Lowest eigenvalue of T_m (diag a[0..m), off-diagonal b[1..m)) by one wave:
// each round evaluates 64 points of the bracket and keeps the sub-interval
// holding the first eigenvalue.  Result valid in every lane of the wave.
__device__ double wave_lowest(const double* a, const double* b, int m) {
  const int lane = threadIdx.x & 63;
  double lo = 1e300, hi = -1e300;
  for (int i = lane; i < m; i += 64) {
    const double r = (i > 0 ? fabs(b[i]) : 0.0) + (i + 1 < m ? fabs(b[i + 1]) : 0.0);
    lo = fmin(lo, a[i] - r);
    hi = fmax(hi, a[i] + r);
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    lo = fmin(lo, __shfl_xor(lo, off, 64));
    hi = fmax(hi, __shfl_xor(hi, off, 64));
  }
  const double pad = 1e-14 * fmax(fabs(lo), fabs(hi)) + 1e-300;
  lo -= pad;
  hi += pad;
  for (int round = 0; round < 12; ++round) {
    const double x = lo + (hi - lo) * (double)(lane + 1) / 65.0;
    const int c = sturm(a, b, m, x);
    const unsigned long long mask = __ballot(c >= 1);
    const int first = mask ? __ffsll((long long)mask) - 1 : 64;
    const double nlo = first == 0 ? lo : lo + (hi - lo) * (double)first / 65.0;
    const double nhi = first >= 64 ? hi : lo + (hi - lo) * (double)(first + 1) / 65.0;
    lo = nlo;
    hi = nhi;
    if (hi - lo <= 4e-16 * fmax(fabs(lo), fabs(hi))) break;
  }
  return 0.5 * (lo + hi);
}

// One lane's view: its barrier, partial-sum slots and vectors.
struct LaneCtx {
  unsigned* bar;
  int* err;
  double* pa;        // alpha partials [L]
  double* pn;        // norm partials [L]
  char* lv;          // 3 vectors
  size_t vstride;
  int L, member;
};

// The whole Lanczos recurrence of one job on one lane; returns false if a
// barrier failed (then every member returns).
template <typename T>
__device__ bool solve_job(const BatchJob& J, int jid, BatchOut* __restrict__ out, LaneCtx& C,
                          unsigned& gen, int niter, double tol, int check_every, uint64_t seed,
                          T* amp, T* Wt, double* red, double* ta, double* tb, T* vs) {
  const int tid = threadIdx.x;
  const int wave = tid >> 6;
  const int wl = tid & 63;
  const T* __restrict__ eup = static_cast<const T*>(J.eup);
  const T* __restrict__ edw = static_cast<const T*>(J.edw);
  __syncthreads();
  for (int i = tid; i < kAmpTable; i += kThreads) amp[i] = static_cast<const T*>(J.amp)[i];
  for (int i = tid; i < 64; i += kThreads) Wt[i] = static_cast<const T*>(J.W)[i];
  const int64_t dup = J.dup, ddw = J.ddw, D = dup * ddw;
  const int L = C.L;
  const int64_t gstride = (int64_t)L * kThreads;
  const int64_t gbase = (int64_t)C.member * kThreads + tid;
  T* buf[3] = {reinterpret_cast<T*>(C.lv), reinterpret_cast<T*>(C.lv + C.vstride),
               reinterpret_cast<T*>(C.lv + 2 * C.vstride)};

  // start vector u_0 and |u_0|^2
  double acc = 0.0;
  for (int64_t i = gbase; i < D; i += gstride) {
    const uint64_t z = splitmix64(seed, (uint64_t)i);
    const T t = (T)((double)(z >> 11) * 0x1.0p-53 * 2.0 - 1.0);
    buf[0][i] = t;
    acc += (double)t * (double)t;
  }
  {
    const double s = block_sum(acc, red);
    if (tid == 0) C.pn[C.member] = s;
  }
  if (!lane_barrier(C.bar, gen, L, C.err)) return false;
  double nrm2 = 0.0;
  for (int m = 0; m < L; ++m) nrm2 += C.pn[m];
  double sc_cur = 1.0 / sqrt(nrm2), sc_prev = 0.0, beta_j = 0.0;
  if (tid == 0) tb[0] = 0.0;
  __syncthreads();
  int steps = 0, status = 4, bdown = 0;
  double E = 0.0, Eold = 0.0, tnorm = 0.0, blast = 0.0;
  const int64_t nslab = (dup + 63) / 64;
  const int64_t nchunk = (ddw + J.rcols - 1) / J.rcols;
  const int64_t nrow_items = nslab * nchunk;
  const int64_t ncol_items = (ddw + J.ccols - 1) / J.ccols;
  const int64_t rbeg = C.member, rend = nrow_items, rstep = L;

  for (int j = 0; j < niter; ++j) {
    const T* cur = buf[j % 3];
    const T* prv = buf[(j + 2) % 3];
    T* w = buf[(j + 1) % 3];
    const T scj = (T)sc_cur;
    // ---- row pass: w = (1 (x) H_dw)(s_j u_j); a wave covers 64 rows of a column
    for (int64_t item = rbeg; item < rend; item += rstep) {
      const int64_t slab = item / nchunk;
      const int64_t jb = (item - slab * nchunk) * J.rcols;
      const int64_t je = min(jb + (int64_t)J.rcols, ddw);
      const int64_t iu = slab * 64 + wl;
      const bool ok = iu < dup;
      const int64_t iuc = ok ? iu : 0;
      for (int64_t c = jb + wave; c < je; c += kWaves) {
        const int64_t cu = __builtin_amdgcn_readfirstlane((int)c);
        T s2 = T(0);
        for (int k0 = 0; k0 < J.sdw; k0 += 8) {
          uint32_t e[8];
#pragma unroll
          for (int k = 0; k < 8; ++k) e[k] = J.hdw[cu * J.sdw + k0 + k];
          T g[8];
#pragma unroll
          for (int k = 0; k < 8; ++k) g[k] = cur[iuc + (int64_t)(e[k] & kColMask) * dup];
#pragma unroll
          for (int k = 0; k < 8; ++k) s2 += amp[e[k] >> kAmpShift] * g[k];
        }
        if (ok) __builtin_nontemporal_store(s2 * scj, w + iu + cu * dup);
      }
    }
    if (!lane_barrier(C.bar, gen, L, C.err)) return false;
    // ---- column pass: w += (H_d + H_up (x) 1)(s_j u_j); <v_j, w> partial.
    // A thread owns a row and reads its hop list once for all staged columns.
    acc = 0.0;
    for (int64_t g0 = C.member; g0 < ncol_items; g0 += L) {
      const int64_t j0 = g0 * J.ccols;
      const int nc = (int)min((int64_t)J.ccols, ddw - j0);
      const int64_t n = (int64_t)nc * dup;
      __syncthreads();
      {
        const T* src = cur + j0 * dup;
        int64_t i = tid;
        for (; i + 3 * kThreads < n; i += 4 * kThreads) {
          const T x0 = src[i], x1 = src[i + kThreads], x2 = src[i + 2 * kThreads],
                  x3 = src[i + 3 * kThreads];
          vs[i] = x0 * scj;
          vs[i + kThreads] = x1 * scj;
          vs[i + 2 * kThreads] = x2 * scj;
          vs[i + 3 * kThreads] = x3 * scj;
        }
        for (; i < n; i += kThreads) vs[i] = src[i] * scj;
      }
      __syncthreads();
      for (int64_t iu = tid; iu < dup; iu += kThreads) {
        T wold[kColMaxB];
#pragma unroll
        for (int c = 0; c < kColMaxB; ++c) wold[c] = c < nc ? w[iu + (j0 + c) * dup] : T(0);
        const T eu = eup[iu];
        const int pu = J.pup[iu] * 8;
        T a4[kColMaxB];
#pragma unroll
        for (int c = 0; c < kColMaxB; ++c) a4[c] = T(0);
        for (int k0 = 0; k0 < J.sup; k0 += 8) {
          uint32_t e[8];
          const uint4* ep = reinterpret_cast<const uint4*>(J.hup + iu * J.sup + k0);
          const uint4 x = ep[0], y = ep[1];
          e[0] = x.x; e[1] = x.y; e[2] = x.z; e[3] = x.w;
          e[4] = y.x; e[5] = y.y; e[6] = y.z; e[7] = y.w;
#pragma unroll
          for (int k = 0; k < 8; ++k) {
            const T am = amp[e[k] >> kAmpShift];
            const int64_t col = e[k] & kColMask;
#pragma unroll
            for (int c = 0; c < kColMaxB; ++c)
              if (c < nc) a4[c] += am * vs[c * dup + col];
          }
        }
#pragma unroll
        for (int c = 0; c < kColMaxB; ++c) {
          if (c >= nc) break;
          const int64_t jj = j0 + c;
          const T xv = vs[c * dup + iu];
          const T r = a4[c] + (eu + edw[jj] + Wt[pu + J.pdw[jj]]) * xv + wold[c];
          w[iu + jj * dup] = r;
          acc += (double)xv * (double)r;
        }
      }
    }
    {
      const double s = block_sum(acc, red);
      if (tid == 0) C.pa[C.member] = s;
    }
    if (!lane_barrier(C.bar, gen, L, C.err)) return false;
    double alpha = 0.0;
    for (int m = 0; m < L; ++m) alpha += C.pa[m];
    // ---- update: w -= alpha v_j + beta_j v_{j-1}; |w|^2 partial
    const double ac = alpha * sc_cur, bc = beta_j * sc_prev;
    acc = 0.0;
    for (int64_t i = gbase; i < D; i += gstride) {
      double r = (double)w[i] - ac * (double)cur[i];
      if (j > 0) r -= bc * (double)prv[i];
      const T t = (T)r;
      w[i] = t;
      acc += (double)t * (double)t;
    }
    {
      const double s = block_sum(acc, red);
      if (tid == 0) C.pn[C.member] = s;
    }
    if (!lane_barrier(C.bar, gen, L, C.err)) return false;
    nrm2 = 0.0;
    for (int m = 0; m < L; ++m) nrm2 += C.pn[m];
    const double bnext = sqrt(nrm2);
    if (tid == 0) {
      ta[j] = alpha;
      tb[j + 1] = bnext;
    }
    __syncthreads();
    steps = j + 1;
    blast = bnext;
    tnorm = fmax(tnorm, fabs(alpha) + beta_j + bnext);
    const bool bd = !(bnext > 1e-12 * tnorm);
    const bool check = bd || (j + 1) % check_every == 0 || j + 1 == niter;
    if (check) {
      if (wave == 0) {
        const double e1 = wave_lowest(ta, tb, j + 1);
        const double e0 = j > 0 ? wave_lowest(ta, tb, j) : e1 + 1.0;
        if (tid == 0) {
          red[0] = e1;
          red[1] = e0;
        }
      }
      __syncthreads();
      E = red[0];
      Eold = red[1];
      __syncthreads();
      const double floor32 = sizeof(T) == 4 ? 2.0 * 1.1920929e-7 * tnorm : 0.0;
      const bool conv = j > 0 && fabs(E - Eold) <= fmax(tol * fmax(1.0, fabs(E)), floor32);
      if (conv || bd) {
        status = 0;
        bdown = bd ? 1 : 0;
        break;
      }
    }
    sc_prev = sc_cur;
    sc_cur = bnext > 0.0 ? 1.0 / bnext : 0.0;
    beta_j = bnext;
  }
  if (C.member == 0 && tid == 0) {
    out[jid].e0 = E;
    out[jid].beta_last = blast;
    out[jid].iters = steps;
    out[jid].status = status;
    out[jid].breakdown = bdown;
  }
  return true;
}

// Jobs [0, njobs) on lanes of L workgroups inside one XCD.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_batch(
    const BatchJob* __restrict__ jobs, int njobs, BatchOut* __restrict__ out,
    unsigned* __restrict__ ctl, int* __restrict__ slots, int* __restrict__ err,
    double* __restrict__ parts, char* __restrict__ vecs, size_t vstride, int L,
    int lanes_per_xcd, int niter, double tol, int check_every, uint64_t seed) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* amp = reinterpret_cast<T*>(smem_raw);
  T* Wt = amp + kAmpTable;
  double* red = reinterpret_cast<double*>(Wt + 64);
  double* ta = red + kWaves;           // alpha[0..niter]
  double* tb = ta + (niter + 2);       // beta[0..niter+1]; tb[j] couples j-1 and j
  __shared__ int s_job;
  T* vs = reinterpret_cast<T*>(tb + (niter + 2));
  const int b = blockIdx.x;
  const int tid = threadIdx.x;
  unsigned* queue = ctl;
  unsigned* bars = ctl + 1;            // one per lane
  const int xcd = b & 7;
  const int in_xcd = b >> 3;
  const int lane = xcd * lanes_per_xcd + in_xcd / L;
  const int member = in_xcd % L;
  double* pa = parts + (size_t)lane * 2 * L;
  LaneCtx C{bars + lane, err, pa, pa + L, vecs + (size_t)lane * 3 * vstride, vstride, L, member};
  unsigned gen = 0;
  for (;;) {
    if (member == 0 && tid == 0) slots[lane] = (int)atomicAdd(queue, 1u);
    if (!lane_barrier(C.bar, gen, L, err)) return;
    if (tid == 0) s_job = __hip_atomic_load(slots + lane, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    const int jid = s_job;
    if (jid >= njobs) return;
    if (!solve_job<T>(jobs[jid], jid, out, C, gen, niter, tol, check_every, seed, amp, Wt, red, ta,
                      tb, vs))
      return;
  }
}

}  // namespace

size_t batch_workspace_bytes(const edx_sector* const* secs, int n, int vtype, int L,
                             int64_t wide_min);
int64_t batch_wide_default();

size_t batch_lds_bytes(int vtype, int64_t max_cols_elems, int niter) {
  const size_t sz = vbytes(vtype);
  return kAmpTable * sz + 64 * sz + kWaves * 8 + 2 * (size_t)(niter + 2) * 8 +
         (size_t)max_cols_elems * sz + 64;
}

namespace {

struct BatchLayout {
  size_t o_jobs, o_out, o_ctl, o_parts, o_wide, o_vec, total;
  size_t wide_bytes, vstride;
  int nlanes, lanes_per_xcd;
};

// wide_ws: plain Lanczos workspace of the largest job run through the
// whole-GPU path (0 if none), one per stream; dmax_narrow: largest dimension
// run in lanes
BatchLayout batch_layout(int n, int vtype, int L, int ncu, size_t wide_ws, int64_t dmax_narrow) {
  BatchLayout B{};
  const size_t sz = vbytes(vtype);
  B.lanes_per_xcd = std::max(1, ncu / 8 / L);
  B.nlanes = 8 * B.lanes_per_xcd;
  B.wide_bytes = wide_ws;
  B.vstride = align_up((size_t)std::max<int64_t>(dmax_narrow, 1) * sz);
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t o2 = off; off += align_up(bytes); return o2; };
  B.o_jobs = take(sizeof(BatchJob) * n);
  B.o_out = take(sizeof(BatchOut) * n);
  // ctl: [queue, barrier per lane], slots [nlanes], err
  B.o_ctl = take(sizeof(unsigned) * (1 + B.nlanes) + sizeof(int) * (1 + B.nlanes) + 64);
  B.o_parts = take(sizeof(double) * (2 * (size_t)L * B.nlanes));
  B.o_wide = take(align_up(wide_ws) * kWideStreams);
  B.o_vec = take(dmax_narrow > 0 ? B.vstride * 3 * B.nlanes : 0);
  B.total = off + 256;
  return B;
}

int device_cus() {
  int dev = 0, ncu = 256;
  if (hipGetDevice(&dev) == hipSuccess) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess) ncu = prop.multiProcessorCount;
  }
  return ncu;
}

}  // namespace

int64_t batch_wide_default() { return 2000000; }

// Jobs of the whole-GPU path: D >= wide_min, and every sector with spin
// exchange, pair hopping or phonons (the lanes implement the spin-separable
// electronic H only).
static bool is_wide(const edx_sector* s, int64_t wide_min) {
  return s->nd || s->dph > 1 || (wide_min > 0 && s->dim >= wide_min);
}

// Work units of the whole-GPU path: jobs of one shape grouped K at a time for
// the multi-set pass (K the largest of 8, 4, 2 not above multi_k that the
// shape supports and that the group fills; shapes up to kMultiMaxDim states),
// the rest one by one; the order is by decreasing dimension.
std::vector<std::vector<int>> wide_units(const edx_sector* const* secs, const std::vector<int>& wide,
                                         int vtype, int multi_k) {
  std::vector<std::vector<int>> units;
  std::vector<char> used(wide.size(), 0);
  for (size_t a = 0; a < wide.size(); ++a) {
    if (used[a]) continue;
    const edx_sector* s = secs[wide[a]];
    std::vector<int> same;
    for (size_t b = a; b < wide.size(); ++b)
      if (!used[b] && multi_same_shape(s, secs[wide[b]])) same.push_back((int)b);
    size_t pos = 0;
    for (int K : {8, 4, 2}) {
      if (K > multi_k || (vtype == EDX_F64 && K > kMultiMaxF64) || s->dim > kMultiMaxDim ||
          !multi_supported(s, K, vtype))
        continue;
      while (same.size() - pos >= (size_t)K) {
        std::vector<int> u;
        for (int q = 0; q < K; ++q) {
          u.push_back(wide[same[pos + q]]);
          used[same[pos + q]] = 1;
        }
        units.push_back(u);
        pos += K;
      }
    }
    for (; pos < same.size(); ++pos) {
      units.push_back({wide[same[pos]]});
      used[same[pos]] = 1;
    }
  }
  std::stable_sort(units.begin(), units.end(), [&](const std::vector<int>& x,
                                                   const std::vector<int>& y) {
    return secs[x[0]]->dim * (int64_t)x.size() > secs[y[0]]->dim * (int64_t)y.size();
  });
  return units;
}

size_t wide_unit_bytes(const edx_sector* const* secs, const std::vector<int>& u, int vtype,
                       int niter) {
  if (u.size() == 1) return lanczos_workspace_bytes(secs[u[0]], vtype, niter, 0);
  return multi_workspace_bytes(secs[u[0]], (int)u.size(), vtype, niter);
}

edx_status batch_run(const edx_sector* const* secs, int n, const edx_lanczos_opts* o,
                     const int* ccols, const int* rcols, int L, int64_t wide_min, int multi_k,
                     void* ws, size_t ws_bytes, edx_batch_result* res, hipStream_t st,
                     double* elapsed_ms) {
  if (n <= 0) return EDX_OK;
  if (multi_k == 0) multi_k = kMultiDefault;
  const int vtype = o->vtype;
  const int ncu = device_cus();
  if (ncu % 8 != 0 || (ncu / 8) % L != 0) {
    set_error("batch: lane size must divide the CUs per XCD");
    return EDX_E_INVALID;
  }
  if (wide_min == 0) wide_min = batch_wide_default();
  // job order by decreasing D: the whole-GPU jobs (D >= wide_min) first, then
  // the lane jobs, which lanes take from the queue largest first
  std::vector<int> order(n);
  for (int i = 0; i < n; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
    const bool wx = is_wide(secs[x], wide_min), wy = is_wide(secs[y], wide_min);
    return wx != wy ? wx : secs[x]->dim > secs[y]->dim;
  });
  int nwide = 0;
  size_t wide_ws = 0;
  int64_t dmax_n = 0, colmax = 1;
  std::vector<int> wide;
  for (int k = 0; k < n; ++k) {
    const edx_sector* s = secs[order[k]];
    if (is_wide(s, wide_min)) {
      ++nwide;
      wide.push_back(order[k]);
    } else {
      dmax_n = std::max(dmax_n, s->dim);
    }
  }
  const std::vector<std::vector<int>> units = wide_units(secs, wide, vtype, multi_k);
  for (const auto& u : units) wide_ws = std::max(wide_ws, wide_unit_bytes(secs, u, vtype, o->niter));
  const int nl = n - nwide;
  std::vector<BatchJob> jobs(nl);
  for (int k = 0; k < nl; ++k) {
    const edx_sector* s = secs[order[nwide + k]];
    BatchJob& J = jobs[k];
    J.hup = s->up.hop;
    J.hdw = s->dw.hop;
    J.eup = vtype == EDX_F32 ? (const void*)s->up.e32 : (const void*)s->up.e64;
    J.edw = vtype == EDX_F32 ? (const void*)s->dw.e32 : (const void*)s->dw.e64;
    J.pup = s->up.pat;
    J.pdw = s->dw.pat;
    J.amp = vtype == EDX_F32 ? (const void*)s->amp32 : (const void*)s->amp64;
    J.W = vtype == EDX_F32 ? (const void*)s->w32 : (const void*)s->w64;
    J.dup = s->dup;
    J.ddw = s->ddw;
    J.sup = s->up.wpad;
    J.sdw = s->dw.wpad;
    J.ccols = std::min(kColMaxB, std::max(1, ccols ? ccols[order[nwide + k]] : 1));
    J.rcols = std::max(1, rcols ? rcols[order[nwide + k]] : 32);
    colmax = std::max(colmax, (int64_t)J.ccols * s->dup);
  }
  const size_t lds = batch_lds_bytes(vtype, colmax, o->niter);
  if (nl > 0 && lds > 160 * 1024) {
    set_error("batch: columns per item do not fit in LDS");
    return EDX_E_UNSUPPORTED;
  }
  const BatchLayout B = batch_layout(nl, vtype, L, ncu, wide_ws, dmax_n);
  char* base = reinterpret_cast<char*>(align_up(reinterpret_cast<uintptr_t>(ws)));
  if (B.total > ws_bytes) {
    set_error("batch: workspace too small (need " + std::to_string(B.total) + " bytes)");
    return EDX_E_NOMEM;
  }
  hipEvent_t e0, e1;
  EDX_HIP(hipEventCreate(&e0));
  EDX_HIP(hipEventCreate(&e1));
  EDX_HIP(hipEventRecord(e0, st));
  // whole-GPU jobs: the plain recurrence and stop rule, largest first, on
  // kWideStreams streams (the caller's and ones created here)
  if (nwide > 0) {
    edx_lanczos_opts q = *o;
    q.reorth = 0;
    q.start = nullptr;   // every job starts from its own SplitMix64 vector
    // helper threads start on device 0: they are given the caller's device
    int dev = 0;
    EDX_HIP(hipGetDevice(&dev));
    const int nst = std::min(kWideStreams, (int)units.size());
    std::vector<hipStream_t> sts(nst, st);
    std::vector<hipEvent_t> done(nst, nullptr);
    edx_status fail = EDX_OK;
    for (int t = 1; t < nst && fail == EDX_OK; ++t) {
      if (hipStreamCreateWithFlags(&sts[t], hipStreamNonBlocking) != hipSuccess ||
          hipEventCreateWithFlags(&done[t], hipEventDisableTiming) != hipSuccess ||
          hipStreamWaitEvent(sts[t], e0, 0) != hipSuccess) {
        set_error("batch: stream set-up failed");
        fail = EDX_E_DEVICE;
      }
    }
    std::atomic<int> next{0};
    const int nunits = (int)units.size();
    std::vector<edx_status> tst(nst, EDX_OK);
    std::vector<std::string> terr(nst);
    auto worker = [&](int t) {
      if (t > 0 && hipSetDevice(dev) != hipSuccess) {
        tst[t] = EDX_E_DEVICE;
        terr[t] = "batch: hipSetDevice failed in a helper thread";
        next.store(nunits);
        return;
      }
      char* wsp = base + B.o_wide + (size_t)t * align_up(B.wide_bytes);
      for (;;) {
        const int k = next.fetch_add(1);
        if (k >= nunits) break;
        const std::vector<int>& u = units[k];
        if (u.size() > 1) {
          // one shape, several bath sets: the multi-set pass
          std::vector<const edx_sector*> g;
          for (int id : u) g.push_back(secs[id]);
          std::vector<edx_batch_result> rr(u.size());
          const edx_status sg = multi_ground_states(g.data(), (int)u.size(), &q, wsp,
                                                    B.wide_bytes, rr.data(), sts[t]);
          if (sg != EDX_OK) {
            tst[t] = sg;
            terr[t] = std::string("batch: multi-set group: ") + edx_last_error();
            next.store(nunits);
            break;
          }
          for (size_t b = 0; b < u.size(); ++b) res[u[b]] = rr[b];
          continue;
        }
        const edx_sector* s = secs[u[0]];
        double e = 0.0;
        edx_lanczos_report rep{};
        const edx_status sj =
            lanczos_ground_state_impl(s, &q, wsp, B.wide_bytes, &e, nullptr, &rep, sts[t]);
        if (sj != EDX_OK && sj != EDX_E_NOCONV && sj != EDX_E_DEGENERATE) {
          tst[t] = sj;
          terr[t] = std::string("batch: whole-GPU job: ") + edx_last_error();
          next.store(nunits);
          break;
        }
        edx_batch_result& r = res[u[0]];
        r.e0 = e;
        r.beta_last = rep.beta_last;
        r.iters = rep.iters;
        r.status = sj == EDX_E_NOCONV ? EDX_E_NOCONV : EDX_OK;
        r.breakdown = rep.breakdown;
      }
    };
    if (fail == EDX_OK) {
      std::vector<std::thread> th;
      for (int t = 1; t < nst; ++t) th.emplace_back(worker, t);
      worker(0);
      for (auto& x : th) x.join();
    }
    // the caller's stream continues after every helper stream's work
    for (int t = 1; t < nst; ++t) {
      if (done[t] && sts[t] != st) {
        (void)hipEventRecord(done[t], sts[t]);
        (void)hipStreamWaitEvent(st, done[t], 0);
      }
    }
    for (int t = 1; t < nst; ++t) {
      if (sts[t] != st) (void)hipStreamSynchronize(sts[t]);
      if (done[t]) (void)hipEventDestroy(done[t]);
      if (sts[t] != st) (void)hipStreamDestroy(sts[t]);
    }
    for (int t = 0; t < nst && fail == EDX_OK; ++t)
      if (tst[t] != EDX_OK) {
        fail = tst[t];
        set_error(terr[t]);
      }
    if (fail != EDX_OK) {
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      return fail;
    }
  }
  int herr = 0;
  std::vector<BatchOut> hout(nl);
  if (nl > 0) {
    BatchJob* d_jobs = reinterpret_cast<BatchJob*>(base + B.o_jobs);
    BatchOut* d_out = reinterpret_cast<BatchOut*>(base + B.o_out);
    unsigned* d_ctl = reinterpret_cast<unsigned*>(base + B.o_ctl);
    int* d_slots = reinterpret_cast<int*>(d_ctl + 1 + B.nlanes);
    int* d_err = d_slots + B.nlanes;
    double* d_parts = reinterpret_cast<double*>(base + B.o_parts);
    char* d_vec = base + B.o_vec;
    EDX_HIP(hipMemcpyAsync(d_jobs, jobs.data(), sizeof(BatchJob) * nl, hipMemcpyHostToDevice, st));
    EDX_HIP(hipMemsetAsync(d_out, 0, sizeof(BatchOut) * nl, st));
    EDX_HIP(hipMemsetAsync(d_ctl, 0, sizeof(unsigned) * (1 + B.nlanes) + sizeof(int) * (1 + B.nlanes),
                           st));
    int niter = o->niter;
    double tol = o->tol;
    int every = std::max(1, o->check_every);
    uint64_t seed = o->seed;
    int njobs = nl;
    size_t vs = B.vstride;
    int lpx = B.lanes_per_xcd;
    void* args[] = {&d_jobs, &njobs, &d_out, &d_ctl, &d_slots, &d_err, &d_parts, &d_vec,
                    &vs, &L, &lpx, &niter, &tol, &every, &seed};
    const void* kern =
        vtype == EDX_F32 ? (const void*)k_batch<float> : (const void*)k_batch<double>;
    EDX_HIP(hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    int per_cu = 0;
    EDX_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, kThreads, lds));
    if (per_cu < 1) {
      set_error("batch: kernel does not fit on a CU");
      return EDX_E_UNSUPPORTED;
    }
    EDX_HIP(hipLaunchCooperativeKernel(kern, dim3(ncu), dim3(kThreads), args, lds, st));
    EDX_HIP(hipMemcpyAsync(hout.data(), d_out, sizeof(BatchOut) * nl, hipMemcpyDeviceToHost, st));
    EDX_HIP(hipMemcpyAsync(&herr, d_err, sizeof(int), hipMemcpyDeviceToHost, st));
  }
  EDX_HIP(hipEventRecord(e1, st));
  EDX_HIP(hipStreamSynchronize(st));
  float ms = 0.f;
  EDX_HIP(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (elapsed_ms) *elapsed_ms = ms;
  for (int k = 0; k < nl; ++k) {
    edx_batch_result& r = res[order[nwide + k]];
    r.e0 = hout[k].e0;
    r.beta_last = hout[k].beta_last;
    r.iters = hout[k].iters;
    r.status = herr ? EDX_E_DEVICE : hout[k].status;
    r.breakdown = hout[k].breakdown;
  }
  if (herr) {
    set_error("batch: a lane barrier timed out");
    return EDX_E_DEVICE;
  }
  return EDX_OK;
}

// Autotuner: for every distinct (D_up, D_dw) among the jobs, time a short run
// (a few Lanczos steps, no stop rule) of up to 8 such jobs on lanes with each
// candidate (columns per column item, columns per row item) and keep the
// fastest; then time the whole batch with each lane size and each threshold
// for the whole-GPU path.
edx_status batch_autotune(const edx_sector* const* secs, int n, const edx_lanczos_opts* o,
                          void* ws, size_t ws_bytes, int* ccols, int* rcols, int* lane_wgs,
                          int64_t* wide_min, hipStream_t st) {
  edx_lanczos_opts q = *o;
  q.start = nullptr;
  q.niter = 6;
  q.tol = 0.0;
  q.check_every = 1000;
  const size_t sz = vbytes(o->vtype);
  std::vector<edx_batch_result> res(n);
  // group jobs by shape
  std::vector<std::pair<std::pair<int64_t, int64_t>, std::vector<int>>> classes;
  for (int i = 0; i < n; ++i) {
    const auto key = std::make_pair(secs[i]->dup, secs[i]->ddw);
    auto it = std::find_if(classes.begin(), classes.end(),
                           [&](const auto& c) { return c.first == key; });
    if (it == classes.end()) {
      classes.push_back({key, {i}});
    } else {
      it->second.push_back(i);
    }
  }
  int L = 32;
  for (auto& cl : classes) {
    const int64_t dup = cl.first.first;
    std::vector<const edx_sector*> sub;
    for (int i : cl.second) {
      if ((int)sub.size() >= 8) break;
      sub.push_back(secs[i]);
    }
    double best = 1e300;
    int bc = 1, br = 32;
    for (int cc : {1, 2, 3, 4}) {
      if (batch_lds_bytes(o->vtype, (int64_t)cc * dup, q.niter) > 150 * 1024) continue;
      for (int rc : {16, 32, 64}) {
        std::vector<int> c1(sub.size(), cc), r1(sub.size(), rc);
        double ms = 0;
        EDX_TRY(batch_run(sub.data(), (int)sub.size(), &q, c1.data(), r1.data(), L, -1, 1, ws,
                          ws_bytes, res.data(), st, &ms));
        if (ms < best) {
          best = ms;
          bc = cc;
          br = rc;
        }
      }
    }
    (void)sz;
    for (int i : cl.second) {
      ccols[i] = bc;
      rcols[i] = br;
    }
  }
  double best = 1e300;
  int bl = 32;
  int64_t bw = batch_wide_default();
  for (int64_t wm : {(int64_t)-1, (int64_t)250000, (int64_t)1000000, batch_wide_default(),
                     (int64_t)4000000, (int64_t)8000000})
    for (int l : {8, 16, 32}) {
      if (batch_workspace_bytes(secs, n, o->vtype, l, wm) > ws_bytes) continue;
      double ms = 0;
      EDX_TRY(batch_run(secs, n, &q, ccols, rcols, l, wm, 0, ws, ws_bytes, res.data(), st, &ms));
      if (ms < best) {
        best = ms;
        bl = l;
        bw = wm;
      }
    }
  *lane_wgs = bl;
  *wide_min = bw;
  return EDX_OK;
}

size_t batch_workspace_bytes(const edx_sector* const* secs, int n, int vtype, int L,
                             int64_t wide_min) {
  if (wide_min == 0) wide_min = batch_wide_default();
  size_t ww = 0;
  int64_t dn = 0;
  int nl = 0;
  std::vector<int> wide;
  for (int i = 0; i < n; ++i) {
    if (is_wide(secs[i], wide_min)) {
      wide.push_back(i);
    } else {
      dn = std::max(dn, secs[i]->dim);
      ++nl;
    }
  }
  // enough for every grouping up to the largest multi-set group
  for (const auto& u : wide_units(secs, wide, vtype, 8))
    ww = std::max(ww, wide_unit_bytes(secs, u, vtype, kMaxBatchIter));
  for (int i : wide) ww = std::max(ww, lanczos_workspace_bytes(secs[i], vtype, kMaxBatchIter, 0));
  return batch_layout(nl, vtype, L, device_cus(), ww, dn).total;
}

}  // namespace edx
