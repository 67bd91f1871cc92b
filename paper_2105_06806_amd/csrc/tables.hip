// Sector tables on the device: string map and rank, per-spin hopping lists with
// fermionic signs, and the diagonal ("popcount") tables.
//
//  * map / rank (Sec. 6 "Sector construction"): the strings of one spin are the
//    Ns-bit integers with popcount N in ascending order.  Instead of scanning and
//    binary-searching, every integer s < 2^Ns computes its position directly as
//    its colex rank sum_k C(c_k, k) over its set bits c_1 < c_2 < ... (ascending
//    integer order of fixed-popcount strings is colex order), so rank[] and
//    map[] come out of one parallel pass and agree with the listing order.
//  * hops (eq. Hbuild, Sec. 2.3): for impurity level a and bath level b > a
//    with exactly one of the two occupied, the neighbour string is
//    s ^ 2^a ^ 2^b and the sign is (-1)^(occupied levels strictly between a and
//    b); the other spin's string never enters because all spin-up modes
//    precede all spin-down modes.  Stored row-major with a padded row length of
//    8, 16 or 24 packed 32-bit entries: column (24 bits) | pair index (7 bits) |
//    sign (1 bit); padding entries point at the row itself with a zero
//    amplitude, so kernels read whole rows without bounds checks.
//  * diagonal (eq. Hbuild, H_d): E_s = sum_k e_k n_k + (U'-J) sum_{a<b} n_a n_b
//    per string and the impurity pattern p = s & (2^norb - 1); the cross-spin
//    terms come from W[p_up][p_dw].
#include <algorithm>
#include <cmath>
#include <cstring>

#include "edx_internal.h"

namespace edx {
namespace {

__global__ void k_rank_map(int ns, int n, const int32_t* __restrict__ binom,
                           int32_t* __restrict__ rank, uint32_t* __restrict__ map) {
  const uint32_t total = 1u << ns;
  for (uint32_t s = blockIdx.x * blockDim.x + threadIdx.x; s < total;
       s += gridDim.x * blockDim.x) {
    if (__popc(s) != n) {
      rank[s] = -1;
      continue;
    }
    int32_t r = 0;
    int k = 1;
    uint32_t x = s;
    while (x) {
      const int c = __ffs(x) - 1;   // lowest set bit
      r += binom[c * (kMaxNs + 1) + k];
      ++k;
      x &= x - 1;
    }
    rank[s] = r;
    map[r] = s;
  }
}

// Orbital-resolved basis (quantum numbers conserved per orbital, Sec. 2.2):
// strings with c[a] electrons among orbital a's levels (its impurity level,
// then its bath levels), indexed as in eq. SectorIndxDecomp: orbital a's
// Nbit-bit string has its colex position r_a among strings with c[a] bits and
// index = sum_a r_a * radix[a], radix[a] = prod_{b<a} C(Nbit, c[b]).
struct OrbCounts {
  int c[kMaxNorb];
  int64_t radix[kMaxNorb];
};

__global__ void k_rank_map_orb(int ns, int norb, int nbath, OrbCounts oc,
                               const int32_t* __restrict__ binom, int32_t* __restrict__ rank,
                               uint32_t* __restrict__ map) {
  const uint32_t total = 1u << ns;
  const uint32_t bmask = nbath >= 32 ? 0xFFFFFFFFu : ((1u << nbath) - 1u);
  for (uint32_t s = blockIdx.x * blockDim.x + threadIdx.x; s < total;
       s += gridDim.x * blockDim.x) {
    int64_t idx = 0;
    bool ok = true;
    for (int a = 0; a < norb && ok; ++a) {
      const uint32_t loc = ((s >> a) & 1u) | (((s >> (norb + a * nbath)) & bmask) << 1);
      if (__popc(loc) != oc.c[a]) {
        ok = false;
        break;
      }
      int32_t r = 0;
      int k = 1;
      uint32_t x = loc;
      while (x) {
        r += binom[(__ffs(x) - 1) * (kMaxNs + 1) + k];
        ++k;
        x &= x - 1;
      }
      idx += (int64_t)r * oc.radix[a];
    }
    rank[s] = ok ? (int32_t)idx : -1;
    if (ok) map[idx] = s;
  }
}

__device__ __forceinline__ int hops_of_row(uint32_t s, int norb, int nbath) {
  int cnt = 0;
  for (int a = 0; a < norb; ++a) {
    const uint32_t na = (s >> a) & 1u;
    for (int nu = 0; nu < nbath; ++nu) {
      const int b = norb + a * nbath + nu;
      cnt += (int)(na ^ ((s >> b) & 1u));
    }
  }
  return cnt;
}

__global__ void k_hop_count(const uint32_t* __restrict__ map, int64_t D, int norb,
                            int nbath, int* __restrict__ width,
                            unsigned long long* __restrict__ nnz) {
  int local_max = 0;
  unsigned long long local_sum = 0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < D;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int c = hops_of_row(map[i], norb, nbath);
    local_max = max(local_max, c);
    local_sum += (unsigned long long)c;
  }
  // integer atomics: order-independent, so the result is deterministic
  atomicMax(width, local_max);
  atomicAdd(nnz, local_sum);
}

__global__ void k_hop_fill(const uint32_t* __restrict__ map,
                           const int32_t* __restrict__ rank, int64_t D, int norb,
                           int nbath, int wpad, uint32_t* __restrict__ hop) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < D;
       i += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t s = map[i];
    int k = 0;
    for (int a = 0; a < norb; ++a) {
      for (int nu = 0; nu < nbath; ++nu) {
        const int p = a * nbath + nu;
        const int b = norb + p;
        if ((((s >> a) ^ (s >> b)) & 1u) == 0u) continue;
        const uint32_t t = s ^ (1u << a) ^ (1u << b);
        const uint32_t between = ((1u << b) - 1u) & ~((2u << a) - 1u);
        const uint32_t sgn = (uint32_t)(__popc(s & between) & 1);
        const uint32_t col = (uint32_t)rank[t];
        hop[i * wpad + k] = col | ((uint32_t)p << kAmpShift) | (sgn << 31);
        ++k;
      }
    }
    for (; k < wpad; ++k) hop[i * wpad + k] = (uint32_t)i | (kPadPair << kAmpShift);
  }
}

__global__ void k_diag(const uint32_t* __restrict__ map, int64_t D, int norb,
                       int ns, const double* __restrict__ elev, double upj,
                       double* __restrict__ e64, float* __restrict__ e32,
                       uint8_t* __restrict__ pat) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < D;
       i += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t s = map[i];
    double e = 0.0;
    for (int k = 0; k < ns; ++k)
      if ((s >> k) & 1u) e += elev[k];
    for (int a = 0; a < norb; ++a)
      for (int b = a + 1; b < norb; ++b)
        if (((s >> a) & (s >> b) & 1u)) e += upj;
    e64[i] = e;
    e32[i] = (float)e;
    pat[i] = (uint8_t)(s & ((1u << norb) - 1u));
  }
}

// Compact spin-up hop rows for the fused pass (D_up < 2^16): per row the wpad
// columns as 16-bit words, then the wpad amplitude indices (entry >> 24) as bytes.
__global__ void k_hrow(const uint32_t* __restrict__ hop, int wpad, int64_t D,
                       uint8_t* __restrict__ out) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < D;
       i += (int64_t)gridDim.x * blockDim.x) {
    uint16_t* c = reinterpret_cast<uint16_t*>(out + i * 3 * wpad);
    uint8_t* x = out + i * 3 * wpad + 2 * wpad;
    for (int k = 0; k < wpad; ++k) {
      const uint32_t f = hop[i * wpad + k];
      c[k] = (uint16_t)(f & 0xFFFFu);
      x[k] = (uint8_t)(f >> kAmpShift);
    }
  }
}

template <typename P>
edx_status dalloc(edx_sector* S, P** p, size_t bytes) {
  bytes = std::max<size_t>(bytes, 1);
  if (S->alloc.alloc) {
    *p = static_cast<P*>(S->alloc.alloc(S->alloc.ctx, bytes));
    if (!*p) {
      set_error("sector tables: allocator out of memory");
      return EDX_E_NOMEM;
    }
    return EDX_OK;
  }
  EDX_HIP(hipMalloc(reinterpret_cast<void**>(p), bytes));
  return EDX_OK;
}

void dfree(edx_sector* S, void* p) {
  if (!p) return;
  if (S->alloc.alloc) {
    if (S->alloc.release) S->alloc.release(S->alloc.ctx, p);
    return;
  }
  (void)hipFree(p);
}

int grid_for(int64_t n, int threads) {
  int64_t b = (n + threads - 1) / threads;
  return (int)std::max<int64_t>(1, std::min<int64_t>(b, 4096));
}

edx_status build_spin(edx_sector* S, SpinTables& T, int n, const int* counts,
                      const double* d_elev, hipStream_t st) {
  const Model& m = S->model;
  T.n = n;
  // C(r, k) from Pascal's triangle
  std::vector<std::vector<int64_t>> C(m.ns + 1, std::vector<int64_t>(m.ns + 1, 0));
  for (int r = 0; r <= m.ns; ++r) {
    C[r][0] = 1;
    for (int k = 1; k <= r; ++k) C[r][k] = C[r - 1][k - 1] + (k <= r - 1 ? C[r - 1][k] : 0);
  }
  int64_t D = C[m.ns][n];
  OrbCounts oc{};
  if (counts) {
    T.orb = true;
    D = 1;
    for (int a = 0; a < m.norb; ++a) {
      T.counts[a] = counts[a];
      oc.c[a] = counts[a];
      oc.radix[a] = D;
      D *= C[m.nbath + 1][counts[a]];
    }
  }
  T.D = D;
  const size_t total = size_t(1) << m.ns;
  EDX_TRY(dalloc(S, &T.rank, total * sizeof(int32_t)));
  EDX_TRY(dalloc(S, &T.map, D * sizeof(uint32_t)));
  if (counts)
    k_rank_map_orb<<<grid_for(total, 256), 256, 0, st>>>(m.ns, m.norb, m.nbath, oc, S->binom,
                                                         T.rank, T.map);
  else
    k_rank_map<<<grid_for(total, 256), 256, 0, st>>>(m.ns, n, S->binom, T.rank, T.map);
  EDX_HIP(hipGetLastError());

  int* d_width = nullptr;
  unsigned long long* d_nnz = nullptr;
  EDX_TRY(dalloc(S, &d_width, sizeof(int) + sizeof(unsigned long long) + 8));
  d_nnz = reinterpret_cast<unsigned long long*>(reinterpret_cast<char*>(d_width) + 8);
  EDX_HIP(hipMemsetAsync(d_width, 0, 16, st));
  k_hop_count<<<grid_for(D, 256), 256, 0, st>>>(T.map, D, m.norb, m.nbath, d_width, d_nnz);
  EDX_HIP(hipGetLastError());
  int width = 0;
  unsigned long long nnz = 0;
  EDX_HIP(hipMemcpyAsync(&width, d_width, sizeof(int), hipMemcpyDeviceToHost, st));
  EDX_HIP(hipMemcpyAsync(&nnz, d_nnz, sizeof(nnz), hipMemcpyDeviceToHost, st));
  EDX_HIP(hipStreamSynchronize(st));
  dfree(S, d_width);
  T.width = width;
  T.wpad = wpad_of(width);
  T.nnz = (int64_t)nnz;
  EDX_TRY(dalloc(S, &T.hop, (size_t)D * T.wpad * sizeof(uint32_t)));
  k_hop_fill<<<grid_for(D, 256), 256, 0, st>>>(T.map, T.rank, D, m.norb, m.nbath, T.wpad, T.hop);
  EDX_HIP(hipGetLastError());
  EDX_TRY(dalloc(S, &T.e64, D * sizeof(double)));
  EDX_TRY(dalloc(S, &T.e32, D * sizeof(float)));
  EDX_TRY(dalloc(S, &T.pat, D));
  k_diag<<<grid_for(D, 256), 256, 0, st>>>(T.map, D, m.norb, m.ns, d_elev,
                                           m.Ust - m.Jh, T.e64, T.e32, T.pat);
  EDX_HIP(hipGetLastError());
  return EDX_OK;
}

void free_spin(edx_sector* S, SpinTables& T) {
  dfree(S, T.map);
  dfree(S, T.rank);
  dfree(S, T.hop);
  dfree(S, T.e64);
  dfree(S, T.e32);
  dfree(S, T.pat);
  T = SpinTables{};
}

}  // namespace

void destroy_sector(edx_sector* s) {
  if (!s) return;
  for (int sp = 0; sp < 2; ++sp)
    for (int k = 0; k < 2; ++k) {
      destroy_sector(s->nb[sp][k]);
      for (int a = 0; a < kMaxNorb; ++a) destroy_sector(s->nb_orb[sp][a][k]);
      destroy_sector(s->nb_pair[sp][k]);
      if (sp == 0) destroy_sector(s->nb_pair[2][k]);
    }
  const bool shared = (s->dw.map == s->up.map);
  free_spin(s, s->up);
  if (!shared) free_spin(s, s->dw);
  dfree(s, s->amp64);
  dfree(s, s->amp32);
  dfree(s, s->hrow);
  dfree(s, s->hrow_dw);
  dfree(s, s->w64);
  dfree(s, s->zeros);
  dfree(s, s->w32);
  dfree(s, s->binom);
  dfree(s, s->corder);
  dfree(s, s->nd_off);
  dfree(s, s->nd_du);
  dfree(s, s->nd_dd);
  dfree(s, s->nd_amp64);
  dfree(s, s->nd_amp32);
  dfree(s, s->ph_off);
  dfree(s, s->ph_du);
  dfree(s, s->ph_dd);
  dfree(s, s->ph_amp64);
  dfree(s, s->ph_amp32);
  dfree(s, s->wph64);
  dfree(s, s->wph32);
  delete s;
}

// Spin exchange X_pq = d+_{p up} d_{p dw} d+_{q dw} d_{q up} (amplitude -Jx)
// and pair hopping P_pq = d+_{p up} d+_{p dw} d_{q dw} d_{q up} (+Jp) of eq.
// Ham1, p != q impurity orbitals, applied to a basis state: whether a term
// acts, its sign and the index shift of the result depend only on the two
// impurity patterns (the lowest norb bits of each spin string).  Sign: the
// operators act right to left on the full string (spin-up modes first), each
// contributing (-1)^(occupied modes below it); both spin-down operators pass
// the same N_up - 1 spin-up electrons, which cancels, leaving per-spin
// parities below impurity levels.  Index shift: a term keeps the number of
// occupied impurity levels of each spin, so every bath bit keeps its position
// in the colex sum sum_k C(c_k, k) and the rank changes by the difference of
// the impurity bits' own terms.
namespace {
int low_rank(uint32_t pat, const std::vector<int32_t>& binom) {
  int r = 0, k = 1;
  for (int c = 0; c < 8; ++c)
    if (pat & (1u << c)) r += binom[c * (kMaxNs + 1) + k++];
  return r;
}
int below(uint32_t s, int m) { return __builtin_popcount(s & ((1u << m) - 1u)) & 1; }
}  // namespace

// H_nd terms per impurity pattern pair (host): off[key]..off[key+1] index the
// (du, dd, amp) of key = pu * P + pd
static void nd_terms_host(const Model& m, const std::vector<int32_t>& binom,
                          std::vector<int32_t>& off, std::vector<int32_t>& du,
                          std::vector<int32_t>& dd, std::vector<double>& amp) {
  const int P = 1 << m.norb;
  off.assign(P * P + 1, 0);
  du.clear();
  dd.clear();
  amp.clear();
  if (!(m.norb >= 2 && (m.Jx != 0.0 || m.Jp != 0.0))) return;
  for (int pu = 0; pu < P; ++pu)
    for (int pd = 0; pd < P; ++pd) {
      for (int p = 0; p < m.norb; ++p)
        for (int q = 0; q < m.norb; ++q) {
          if (p == q) continue;
          const uint32_t bp = 1u << p, bq = 1u << q;
          const uint32_t u = (uint32_t)pu, d = (uint32_t)pd;
          if (m.Jx != 0.0 && (u & bq) && !(u & bp) && (d & bp) && !(d & bq)) {
            const int par = below(u, q) ^ below(d, q) ^ below(d | bq, p) ^ below(u ^ bq, p);
            du.push_back(low_rank((u ^ bq) | bp, binom) - low_rank(u, binom));
            dd.push_back(low_rank((d | bq) ^ bp, binom) - low_rank(d, binom));
            amp.push_back(par ? m.Jx : -m.Jx);
          }
          if (m.Jp != 0.0 && (u & bq) && (d & bq) && !(u & bp) && !(d & bp)) {
            const int par = below(u, q) ^ below(d, q) ^ below(d ^ bq, p) ^ below(u ^ bq, p);
            du.push_back(low_rank((u ^ bq) | bp, binom) - low_rank(u, binom));
            dd.push_back(low_rank((d ^ bq) | bp, binom) - low_rank(d, binom));
            amp.push_back(par ? -m.Jp : m.Jp);
          }
        }
      off[pu * P + pd + 1] = (int32_t)du.size();
    }
}

edx_status build_nd_terms(edx_sector* S, const Model& m, const std::vector<int32_t>& binom,
                          hipStream_t st) {
  std::vector<int32_t> off, du, dd;
  std::vector<double> amp;
  nd_terms_host(m, binom, off, du, dd, amp);
  S->nd_nt = (int)du.size();
  const size_t nt = std::max<size_t>(1, du.size());
  du.resize(nt, 0);
  dd.resize(nt, 0);
  amp.resize(nt, 0.0);
  std::vector<float> ampf(amp.begin(), amp.end());
  EDX_TRY(dalloc(S, &S->nd_off, off.size() * sizeof(int32_t)));
  EDX_TRY(dalloc(S, &S->nd_du, nt * sizeof(int32_t)));
  EDX_TRY(dalloc(S, &S->nd_dd, nt * sizeof(int32_t)));
  EDX_TRY(dalloc(S, &S->nd_amp64, nt * sizeof(double)));
  EDX_TRY(dalloc(S, &S->nd_amp32, nt * sizeof(float)));
  EDX_HIP(hipMemcpyAsync(S->nd_off, off.data(), off.size() * sizeof(int32_t),
                         hipMemcpyHostToDevice, st));
  EDX_HIP(hipMemcpyAsync(S->nd_du, du.data(), nt * sizeof(int32_t), hipMemcpyHostToDevice, st));
  EDX_HIP(hipMemcpyAsync(S->nd_dd, dd.data(), nt * sizeof(int32_t), hipMemcpyHostToDevice, st));
  EDX_HIP(hipMemcpyAsync(S->nd_amp64, amp.data(), nt * sizeof(double), hipMemcpyHostToDevice, st));
  EDX_HIP(hipMemcpyAsync(S->nd_amp32, ampf.data(), nt * sizeof(float), hipMemcpyHostToDevice, st));
  // the host vectors go out of scope: finish the copies first
  EDX_HIP(hipStreamSynchronize(st));
  return EDX_OK;
}

// Per phonon slice p (Sec. "Electron-phonon coupling", eq. HephBuild): the
// coupling G(pu, pd) = sum_a g_a (n_{a up} + n_{a dw}) times sqrt(p) reaches
// slice p - 1 and times sqrt(p + 1) slice p + 1, both at the same electronic
// element, i.e. D_dw columns back or ahead in the vector; merged per pattern
// pair with the H_nd terms so that the fused pass applies both.  W_p = W + w0 p.
static edx_status build_ph_terms(edx_sector* S, const Model& m,
                                 const std::vector<int32_t>& binom, const double* W,
                                 hipStream_t st) {
  const int P = 1 << m.norb, K = P * P, dph = S->dph;
  std::vector<int32_t> noff, ndu, ndd;
  std::vector<double> namp;
  nd_terms_host(m, binom, noff, ndu, ndd, namp);
  std::vector<int32_t> off((size_t)dph * (K + 1), 0), du, dd;
  std::vector<double> amp;
  S->ph_start.assign(dph + 1, 0);
  S->ph_nt_max = 0;
  for (int p = 0; p < dph; ++p) {
    const int start = (int)du.size();
    S->ph_start[p] = start;
    for (int key = 0; key < K; ++key) {
      const int pu = key / P, pd = key % P;
      for (int t = noff[key]; t < noff[key + 1]; ++t) {
        du.push_back(ndu[t]);
        dd.push_back(ndd[t]);
        amp.push_back(namp[t]);
      }
      double G = 0.0;
      for (int a = 0; a < m.norb; ++a) G += m.g[a] * (((pu >> a) & 1) + ((pd >> a) & 1));
      if (G != 0.0) {
        if (p > 0) {
          du.push_back(0);
          dd.push_back((int32_t)-S->ddw);
          amp.push_back(G * std::sqrt((double)p));
        }
        if (p + 1 < dph) {
          du.push_back(0);
          dd.push_back((int32_t)S->ddw);
          amp.push_back(G * std::sqrt((double)(p + 1)));
        }
      }
      off[(size_t)p * (K + 1) + key + 1] = (int32_t)du.size() - start;
    }
    S->ph_nt_max = std::max(S->ph_nt_max, (int)du.size() - start);
  }
  S->ph_start[dph] = (int)du.size();
  const size_t nt = std::max<size_t>(1, du.size());
  du.resize(nt, 0);
  dd.resize(nt, 0);
  amp.resize(nt, 0.0);
  std::vector<float> ampf(amp.begin(), amp.end());
  std::vector<double> wp((size_t)dph * 64);
  std::vector<float> wpf((size_t)dph * 64);
  for (int p = 0; p < dph; ++p)
    for (int k = 0; k < 64; ++k) {
      wp[(size_t)p * 64 + k] = W[k] + m.w0 * p;
      wpf[(size_t)p * 64 + k] = (float)wp[(size_t)p * 64 + k];
    }
  EDX_TRY(dalloc(S, &S->ph_off, off.size() * sizeof(int32_t)));
  EDX_TRY(dalloc(S, &S->ph_du, nt * sizeof(int32_t)));
  EDX_TRY(dalloc(S, &S->ph_dd, nt * sizeof(int32_t)));
  EDX_TRY(dalloc(S, &S->ph_amp64, nt * sizeof(double)));
  EDX_TRY(dalloc(S, &S->ph_amp32, nt * sizeof(float)));
  EDX_TRY(dalloc(S, &S->wph64, wp.size() * sizeof(double)));
  EDX_TRY(dalloc(S, &S->wph32, wpf.size() * sizeof(float)));
  EDX_HIP(hipMemcpyAsync(S->ph_off, off.data(), off.size() * sizeof(int32_t),
                         hipMemcpyHostToDevice, st));
  EDX_HIP(hipMemcpyAsync(S->ph_du, du.data(), nt * sizeof(int32_t), hipMemcpyHostToDevice, st));
  EDX_HIP(hipMemcpyAsync(S->ph_dd, dd.data(), nt * sizeof(int32_t), hipMemcpyHostToDevice, st));
  EDX_HIP(hipMemcpyAsync(S->ph_amp64, amp.data(), nt * sizeof(double), hipMemcpyHostToDevice, st));
  EDX_HIP(hipMemcpyAsync(S->ph_amp32, ampf.data(), nt * sizeof(float), hipMemcpyHostToDevice, st));
  EDX_HIP(hipMemcpyAsync(S->wph64, wp.data(), wp.size() * sizeof(double), hipMemcpyHostToDevice,
                         st));
  EDX_HIP(hipMemcpyAsync(S->wph32, wpf.data(), wpf.size() * sizeof(float), hipMemcpyHostToDevice,
                         st));
  EDX_HIP(hipStreamSynchronize(st));   // host vectors go out of scope
  return EDX_OK;
}

size_t sector_table_bytes(int ns, int nup, int ndw) {
  auto comb = [](int n, int k) -> int64_t {
    if (k < 0 || k > n) return 0;
    int64_t r = 1;
    for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
    return r;
  };
  const size_t a = 256;   // per-allocation alignment slack
  size_t b = 0;
  for (int n : {nup, ndw}) {
    const size_t D = (size_t)comb(ns, n);
    b += ((size_t)4 << ns) + D * (4 + 24 * 4 + 8 + 4 + 1) + 6 * a;
  }
  b += (kMaxNs + 1) * (kMaxNs + 1) * 4 + 256 * 12 + 64 * 12 + 16 + 8 * kMaxNs + 8 * a;
  b += (size_t)comb(ns, ndw) * 4 + a;   // column order
  b += 6 * a + 65 * 4 + 64 * 12 * (4 + 4 + 8 + 4);   // H_nd term table
  b += 8 * ((size_t)std::max(comb(ns, nup), comb(ns, ndw)) + 64) + a;   // zero block
  b += ((size_t)comb(ns, nup) + (size_t)comb(ns, ndw)) * 3 * 24 + 2 * a;   // compact hop rows
  return b;
}

edx_status build_sector_impl(const Model& m, int nup, int ndw, hipStream_t st,
                             edx_sector** out, const Allocator* alloc, const int* cup,
                             const int* cdw) {
  std::unique_ptr<edx_sector, void (*)(edx_sector*)> S(new edx_sector(), destroy_sector);
  if (alloc) S->alloc = *alloc;
  S->model = m;
  S->nup = nup;
  S->ndw = ndw;
  EDX_HIP(hipGetDevice(&S->device));

  // binomial table C(c, k), c, k <= 24
  std::vector<int32_t> binom((kMaxNs + 1) * (kMaxNs + 1), 0);
  for (int c = 0; c <= kMaxNs; ++c) {
    binom[c * (kMaxNs + 1) + 0] = 1;
    for (int k = 1; k <= c; ++k)
      binom[c * (kMaxNs + 1) + k] =
          binom[(c - 1) * (kMaxNs + 1) + k - 1] + (k <= c - 1 ? binom[(c - 1) * (kMaxNs + 1) + k] : 0);
  }
  EDX_TRY(dalloc(S.get(), &S->binom, binom.size() * sizeof(int32_t)));
  EDX_HIP(hipMemcpyAsync(S->binom, binom.data(), binom.size() * sizeof(int32_t),
                         hipMemcpyHostToDevice, st));

  // level energies e_k (impurity shifted by -xmu)
  std::vector<double> elev(m.ns, 0.0);
  for (int a = 0; a < m.norb; ++a) elev[a] = m.eps_imp[a] - m.xmu;
  for (int p = 0; p < m.norb * m.nbath; ++p) elev[m.norb + p] = m.eps_bath[p];
  double* d_elev = nullptr;
  EDX_TRY(dalloc(S.get(), &d_elev, m.ns * sizeof(double)));
  EDX_HIP(hipMemcpyAsync(d_elev, elev.data(), m.ns * sizeof(double),
                         hipMemcpyHostToDevice, st));

  S->orb = cup != nullptr;
  bool same = ndw == nup;
  if (S->orb)
    for (int a = 0; a < m.norb; ++a) same = same && cup[a] == cdw[a];
  edx_status rc = build_spin(S.get(), S->up, nup, cup, d_elev, st);
  if (rc == EDX_OK) {
    if (same) {
      S->dw = S->up;   // identical tables, shared
    } else {
      rc = build_spin(S.get(), S->dw, ndw, cdw, d_elev, st);
    }
  }
  if (rc != EDX_OK) {
    dfree(S.get(), d_elev);
    return rc;
  }
  S->dup = S->up.D;
  S->ddw = S->dw.D;
  S->dph = m.nph + 1;
  S->dim = S->dup * S->ddw * S->dph;
  S->ld = vec_ld(S->dup);
  S->vlen = S->ld * S->ddw * S->dph;
  S->nd = m.norb >= 2 && (m.Jx != 0.0 || m.Jp != 0.0);
  if (S->nd) EDX_TRY(build_nd_terms(S.get(), m, binom, st));

  // column order of the fused H.v pass: spin-down strings stably sorted by
  // impurity pattern (for Norb = 1: impurity empty, then occupied)
  {
    std::vector<uint8_t> pat(S->ddw);
    EDX_HIP(hipMemcpyAsync(pat.data(), S->dw.pat, S->ddw, hipMemcpyDeviceToHost, st));
    EDX_HIP(hipStreamSynchronize(st));
    std::vector<int32_t> ord(S->ddw);
    for (int64_t j = 0; j < S->ddw; ++j) ord[j] = (int32_t)j;
    std::stable_sort(ord.begin(), ord.end(), [&](int32_t x, int32_t y) { return pat[x] < pat[y]; });
    EDX_TRY(dalloc(S.get(), &S->corder, ord.size() * sizeof(int32_t)));
    EDX_HIP(hipMemcpyAsync(S->corder, ord.data(), ord.size() * sizeof(int32_t),
                           hipMemcpyHostToDevice, st));
  }

  // signed amplitude table and pattern interaction table
  double amp[kAmpTable];
  float ampf[kAmpTable];
  for (int idx = 0; idx < kAmpTable; ++idx) {
    const int p = idx & 0x7F;
    const double sg = (idx & 0x80) ? -1.0 : 1.0;
    amp[idx] = (p == (int)kPadPair || p >= m.norb * m.nbath) ? 0.0 : sg * m.vhyb[p];
    ampf[idx] = (float)amp[idx];
  }
  std::memcpy(S->amp_host, amp, sizeof(amp));
  double W[64];
  float Wf[64];
  for (int pu = 0; pu < 8; ++pu)
    for (int pd = 0; pd < 8; ++pd) {
      double w = 0.0;
      for (int a = 0; a < m.norb; ++a) {
        const int na = (pu >> a) & 1;
        w += m.U * na * ((pd >> a) & 1);
        for (int b = 0; b < m.norb; ++b)
          if (a != b) w += m.Ust * na * ((pd >> b) & 1);
      }
      W[pu * 8 + pd] = w;
      Wf[pu * 8 + pd] = (float)w;
    }
  EDX_TRY(dalloc(S.get(), &S->amp64, sizeof(amp)));
  EDX_TRY(dalloc(S.get(), &S->amp32, sizeof(ampf)));
  EDX_TRY(dalloc(S.get(), &S->w64, sizeof(W)));
  EDX_TRY(dalloc(S.get(), &S->w32, sizeof(Wf)));
  EDX_HIP(hipMemcpyAsync(S->amp64, amp, sizeof(amp), hipMemcpyHostToDevice, st));
  EDX_HIP(hipMemcpyAsync(S->amp32, ampf, sizeof(ampf), hipMemcpyHostToDevice, st));
  EDX_HIP(hipMemcpyAsync(S->w64, W, sizeof(W), hipMemcpyHostToDevice, st));
  EDX_HIP(hipMemcpyAsync(S->w32, Wf, sizeof(Wf), hipMemcpyHostToDevice, st));
  // compact hop rows: spin up for the fused pass, spin down for the column
  // pass on the transposed vector
  for (int spin = 0; spin < 2; ++spin) {
    const SpinTables& T = spin == 0 ? S->up : S->dw;
    uint8_t** dst = spin == 0 ? &S->hrow : &S->hrow_dw;
    if (T.D >= 65536) continue;
    EDX_TRY(dalloc(S.get(), dst, (size_t)T.D * 3 * T.wpad));
    hipLaunchKernelGGL(k_hrow, dim3((unsigned)std::min<int64_t>((T.D + 255) / 256, 4096)),
                       dim3(256), 0, st, T.hop, T.wpad, T.D, *dst);
    EDX_HIP(hipGetLastError());
  }
  if (S->dph > 1) EDX_TRY(build_ph_terms(S.get(), m, binom, W, st));
  {
    const size_t zb = sizeof(double) * ((size_t)std::max(S->dup, S->ddw) + 64);
    EDX_TRY(dalloc(S.get(), &S->zeros, zb));
    EDX_HIP(hipMemsetAsync(S->zeros, 0, zb, st));
  }
  EDX_HIP(hipStreamSynchronize(st));
  dfree(S.get(), d_elev);
  *out = S.release();
  return EDX_OK;
}

}  // namespace edx
