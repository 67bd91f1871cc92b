// Green's-function kernels (Sec. 6 "Dynamical correlation functions").
//
//  * k_apply: phi = c+_{orb,s} psi (N_s -> N_s + 1) or c_{orb,s} psi
//    (N_s -> N_s - 1).  One thread per element of the target sector: it looks
//    up the source string through the rank table and copies the amplitude with
//    the fermionic sign (Sec. 2.3): (-1)^(occupied levels below orb of the same
//    spin), times (-1)^N_up for spin down because every spin-up mode precedes
//    the spin-down modes.  The paper applies the operator on the master rank and
//    then scatters the vector; here it is a streaming gather on the device.
//    psi is dense (column stride D_up of the source sector); phi has the
//    padded column stride of the target sector's Krylov vectors, with zeros
//    in the padding rows.
//  * k_cf: the two continued fractions at the Matsubara frequencies
//    w_n = (2n+1) pi / beta, one thread per frequency, evaluated from the
//    deepest level up:
//      d = z -+ (a_{n-1} - E0);  d = z -+ (a_k - E0) - b_{k+1}^2 / d, k = n-2..0;
//      G += w / d    (- for the particle branch, + for the hole branch).
#include "common.h"
#include "edx_internal.h"

namespace edx {
namespace {

template <typename T>
__global__ __launch_bounds__(256) void k_apply(const T* __restrict__ psi, T* __restrict__ phi,
                                               int64_t tdup, int64_t tld, int64_t tddw,
                                               int64_t tlen, int64_t sdup, int64_t sddw,
                                               const uint32_t* __restrict__ tmap,
                                               const int32_t* __restrict__ srank, int orb,
                                               int spin, int create, int nup) {
  const uint32_t bit = 1u << orb;
  const uint32_t below = bit - 1u;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < tlen;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t col = idx / tld;          // column over all phonon slices
    const int64_t iu = idx - col * tld;
    if (iu >= tdup) {
      phi[idx] = T(0);
      continue;
    }
    const int64_t p = col / tddw;           // phonon index (0 without phonons)
    const int64_t id = col - p * tddw;
    const uint32_t t = tmap[spin == 0 ? iu : id];
    const bool has = (t & bit) != 0u;
    T val = T(0);
    if (has == (create != 0)) {
      const uint32_t s = create ? (t ^ bit) : (t | bit);
      const int64_t r = srank[s];
      int par = __popc(s & below) & 1;
      if (spin == 1) par ^= (nup & 1);
      const int64_t src = spin == 0 ? r + (id + p * sddw) * sdup : iu + (r + p * sddw) * sdup;
      const T x = psi[src];
      val = par ? -x : x;
    }
    phi[idx] = val;
  }
}

// phi = (O - mean) psi for O = sum_a (cu[a] n_{a up} + cd[a] n_{a dw}), diagonal
// in the occupation basis, read from the impurity patterns of the two strings.
// psi dense (stride dup), phi padded (stride ld, zero padding).  mean == nullptr:
// only partial sums of <psi|O|psi>; otherwise phi is written and the partial
// sums are |phi|^2.
template <typename T>
__global__ __launch_bounds__(256) void k_diag_op(const T* __restrict__ psi, T* __restrict__ phi,
                                                 int64_t dup, int64_t ld, int64_t ddw,
                                                 int64_t len, const uint8_t* __restrict__ pup,
                                                 const uint8_t* __restrict__ pdw, int norb,
                                                 DiagCoef c, const double* __restrict__ mean,
                                                 double* __restrict__ partial) {
  __shared__ double red[4];
  double acc = 0.0;
  const double mu = mean ? *mean : 0.0;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < len;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t id = idx / ld;
    const int64_t iu = idx - id * ld;
    if (iu >= dup) {
      if (mean) phi[idx] = T(0);
      continue;
    }
    const uint32_t a = pup[iu], b = pdw[id % ddw];   // phonon slices repeat the columns
    double f = 0.0;
    for (int o = 0; o < norb; ++o) f += c.up[o] * ((a >> o) & 1u) + c.dw[o] * ((b >> o) & 1u);
    const double x = (double)psi[iu + id * dup];
    if (mean) {
      const T t = (T)((f - mu) * x);
      phi[idx] = t;
      acc += (double)t * (double)t;
    } else {
      acc += f * x * x;
    }
  }
  const double s = block_sum(acc, red);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// Excitonic operator O = sum_sigma (c+_a c_b + c+_b c_a) (impurity levels a < b,
// same spin): each output string t with exactly one of bits a, b set receives
// psi of t with that electron moved, signed by the occupied levels strictly
// between a and b (unchanged by the move).  Both spins; psi dense, phi padded
// (zero padding); mean == nullptr: only partial sums of <psi|O|psi>; otherwise
// phi = (O - mean) psi and partial sums of |phi|^2.
template <typename T>
__global__ __launch_bounds__(256) void k_exc_op(const T* __restrict__ psi, T* __restrict__ phi,
                                                int64_t dup, int64_t ld, int64_t len,
                                                const uint32_t* __restrict__ umap,
                                                const int32_t* __restrict__ urank,
                                                const uint32_t* __restrict__ dmap,
                                                const int32_t* __restrict__ drank, int a, int b,
                                                const double* __restrict__ mean,
                                                double* __restrict__ partial) {
  __shared__ double red[4];
  const uint32_t mab = (1u << a) | (1u << b);
  const uint32_t between = ((1u << b) - 1u) & ~((2u << a) - 1u);
  const double mu = mean ? *mean : 0.0;
  double acc = 0.0;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < len;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t id = idx / ld;
    const int64_t iu = idx - id * ld;
    if (iu >= dup) {
      if (mean) phi[idx] = T(0);
      continue;
    }
    double val = 0.0;
    const uint32_t tu = umap[iu], td = dmap[id];
    if (__popc(tu & mab) == 1) {
      const double x = (double)psi[urank[tu ^ mab] + id * dup];
      val += (__popc(tu & between) & 1) ? -x : x;
    }
    if (__popc(td & mab) == 1) {
      const double x = (double)psi[iu + (int64_t)drank[td ^ mab] * dup];
      val += (__popc(td & between) & 1) ? -x : x;
    }
    const double x0 = (double)psi[iu + id * dup];
    if (mean) {
      const T t = (T)(val - mu * x0);
      phi[idx] = t;
      acc += (double)t * (double)t;
    } else {
      acc += x0 * val;
    }
  }
  const double s = block_sum(acc, red);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// Pair operators of impurity level a: create = c+_{a up} c+_{a dw} (the spin-down
// creator acts first), else c_{a dw} c_{a up} (the spin-up annihilator first).
// Gather form from the target sector: the source strings are the target's
// with bit a toggled in both spins; the full-string sign counts the occupied
// levels below a of each spin and, for the spin-down operator, every spin-up
// electron present when it acts.
template <typename T>
__global__ __launch_bounds__(256) void k_pair(const T* __restrict__ psi, T* __restrict__ phi,
                                              int64_t tdup, int64_t tld, int64_t tlen,
                                              int64_t sdup, const uint32_t* __restrict__ tumap,
                                              const uint32_t* __restrict__ tdmap,
                                              const int32_t* __restrict__ surank,
                                              const int32_t* __restrict__ sdrank, int a,
                                              int create, int nup_src) {
  const uint32_t bit = 1u << a, below = bit - 1u;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < tlen;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t id = idx / tld;
    const int64_t iu = idx - id * tld;
    if (iu >= tdup) {
      phi[idx] = T(0);
      continue;
    }
    const uint32_t tu = tumap[iu], td = tdmap[id];
    const bool want = create != 0;
    T val = T(0);
    if (((tu & bit) != 0u) == want && ((td & bit) != 0u) == want) {
      const uint32_t su = tu ^ bit, sd = td ^ bit;
      const int nup_dw_op = create ? nup_src : nup_src - 1;   // spin-up count when c_dw acts
      const int par = (__popc(tu & below) + __popc(td & below) + nup_dw_op) & 1;
      const T x = psi[surank[su] + (int64_t)sdrank[sd] * sdup];
      val = par ? -x : x;
    }
    phi[idx] = val;
  }
}

__global__ void k_cf(const double* __restrict__ ap, const double* __restrict__ bp, int np,
                     double wp, const double* __restrict__ ah, const double* __restrict__ bh,
                     int nh, double wh, double e0, double beta, int lmats,
                     double* __restrict__ g, int bosonic) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= lmats) return;
  // fermionic (2n+1) pi / beta, or bosonic 2n pi / beta
  const double wn = (2.0 * n + (bosonic ? 0.0 : 1.0)) * M_PI / beta;
  double gr = 0.0, gi = 0.0;
  for (int br = 0; br < 2; ++br) {
    const double* a = br == 0 ? ap : ah;
    const double* b = br == 0 ? bp : bh;
    const int m = br == 0 ? np : nh;
    const double wgt = br == 0 ? wp : wh;
    const double sg = br == 0 ? -1.0 : 1.0;
    if (m <= 0 || wgt == 0.0) continue;
    // d = z + sg (a_k - e0) - b_{k+1}^2 / d, with z = i wn
    double dr = sg * (a[m - 1] - e0), di = wn;
    for (int k = m - 2; k >= 0; --k) {
      const double b2 = b[k] * b[k];
      const double den = dr * dr + di * di;
      // b2 / d = b2 * conj(d) / |d|^2
      const double qr = b2 * dr / den, qi = -b2 * di / den;
      dr = sg * (a[k] - e0) - qr;
      di = wn - qi;
    }
    const double den = dr * dr + di * di;
    gr += wgt * dr / den;
    gi += -wgt * di / den;
  }
  g[2 * n] = gr;
  g[2 * n + 1] = gi;
}

}  // namespace

edx_status k_apply_op(const edx_sector* src, const edx_sector* dst, int vtype, const void* psi,
                      void* phi, int orb, int spin, int create, hipStream_t st) {
  const int64_t n = dst->vlen;
  const int64_t b = (n + 255) / 256;
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(b, 8192));
  const uint32_t* tmap = spin == 0 ? dst->up.map : dst->dw.map;
  const int32_t* srank = spin == 0 ? src->up.rank : src->dw.rank;
  if (vtype == EDX_F64)
    hipLaunchKernelGGL(k_apply<double>, dim3(grid), dim3(256), 0, st, (const double*)psi,
                       (double*)phi, dst->dup, dst->ld, dst->ddw, n, src->dup, src->ddw, tmap,
                       srank, orb, spin, create, src->nup);
  else
    hipLaunchKernelGGL(k_apply<float>, dim3(grid), dim3(256), 0, st, (const float*)psi,
                       (float*)phi, dst->dup, dst->ld, dst->ddw, n, src->dup, src->ddw, tmap,
                       srank, orb, spin, create, src->nup);
  EDX_HIP(hipGetLastError());
  return EDX_OK;
}

edx_status k_diag_apply(const edx_sector* s, int vtype, const void* psi, void* phi,
                        const DiagCoef& c, const double* mean, double* partial, int nblocks,
                        hipStream_t st) {
  const int64_t n = s->vlen;
  if (vtype == EDX_F64)
    hipLaunchKernelGGL(k_diag_op<double>, dim3(nblocks), dim3(256), 0, st, (const double*)psi,
                       (double*)phi, s->dup, s->ld, s->ddw, n, s->up.pat, s->dw.pat, s->model.norb, c,
                       mean, partial);
  else
    hipLaunchKernelGGL(k_diag_op<float>, dim3(nblocks), dim3(256), 0, st, (const float*)psi,
                       (float*)phi, s->dup, s->ld, s->ddw, n, s->up.pat, s->dw.pat, s->model.norb, c,
                       mean, partial);
  EDX_HIP(hipGetLastError());
  return EDX_OK;
}

edx_status k_exc_apply(const edx_sector* s, int vtype, const void* psi, void* phi, int a,
                       int b, const double* mean, double* partial, int nblocks, hipStream_t st) {
  const int64_t n = s->vlen;
  if (vtype == EDX_F64)
    hipLaunchKernelGGL(k_exc_op<double>, dim3(nblocks), dim3(256), 0, st, (const double*)psi,
                       (double*)phi, s->dup, s->ld, n, s->up.map, s->up.rank, s->dw.map,
                       s->dw.rank, a, b, mean, partial);
  else
    hipLaunchKernelGGL(k_exc_op<float>, dim3(nblocks), dim3(256), 0, st, (const float*)psi,
                       (float*)phi, s->dup, s->ld, n, s->up.map, s->up.rank, s->dw.map,
                       s->dw.rank, a, b, mean, partial);
  EDX_HIP(hipGetLastError());
  return EDX_OK;
}

edx_status k_pair_apply(const edx_sector* src, const edx_sector* dst, int vtype, const void* psi,
                        void* phi, int a, int create, hipStream_t st) {
  const int64_t n = dst->vlen;
  const int64_t b = (n + 255) / 256;
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(b, 8192));
  if (vtype == EDX_F64)
    hipLaunchKernelGGL(k_pair<double>, dim3(grid), dim3(256), 0, st, (const double*)psi,
                       (double*)phi, dst->dup, dst->ld, n, src->dup, dst->up.map, dst->dw.map,
                       src->up.rank, src->dw.rank, a, create, src->nup);
  else
    hipLaunchKernelGGL(k_pair<float>, dim3(grid), dim3(256), 0, st, (const float*)psi,
                       (float*)phi, dst->dup, dst->ld, n, src->dup, dst->up.map, dst->dw.map,
                       src->up.rank, src->dw.rank, a, create, src->nup);
  EDX_HIP(hipGetLastError());
  return EDX_OK;
}

edx_status k_green_cf(const double* ap, const double* bp, int np, double wp, const double* ah,
                      const double* bh, int nh, double wh, double e0, double beta, int lmats,
                      double* g, hipStream_t st, int bosonic) {
  const int grid = (lmats + 255) / 256;
  hipLaunchKernelGGL(k_cf, dim3(grid), dim3(256), 0, st, ap, bp, np, wp, ah, bh, nh, wh, e0,
                     beta, lmats, g, bosonic);
  EDX_HIP(hipGetLastError());
  return EDX_OK;
}

}  // namespace edx
