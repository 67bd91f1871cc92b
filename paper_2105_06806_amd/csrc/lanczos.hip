// Lanczos ground state and Krylov Green's function drivers (host side).
//
// Ground state (Sec. 6 "Diagonalization", plain Lanczos as the paper runs it):
//   alpha_j = <v_j, H v_j>;  w = H v_j - alpha_j v_j - beta_j v_{j-1};
//   beta_{j+1} = |w|;  v_{j+1} = w / beta_{j+1}.
// A step is enqueued without host synchronisation (scalars stay on the
// device); every `check_every` steps the host copies alpha/beta back and
// applies the stop rule:
//   |E_j - E_{j-1}| <= tol max(1, |E_j|)  [and beta_{j+1}|y_j| <= rtol max(1,|E|)],
//   both thresholds floored at 2 eps_32 |T| when the vectors are FP32,
//   or breakdown beta_{j+1} <= 1e-12 max_i(|alpha_i| + beta_i + beta_{i+1}),
//   or j + 1 = niter.
// E_j is the lowest eigenvalue of the tridiagonal T_j (Sturm bisection).  The
// ground vector psi0 = sum_j y_j v_j is formed by replaying the identical
// recurrence (deterministic kernels), so no basis is stored.
//
// Precision mode (vtype = F32): vectors in FP32, all scalars, dot products
// and the tridiagonal problem in FP64; reorth = 1 adds one Gram-Schmidt pass
// against v_j and v_{j-1} per step, reorth = 2 keeps every v_j and applies
// classical Gram-Schmidt twice against all of them.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <limits>

#include "edx_internal.h"

namespace edx {

edx_status k_reduce_strided(const double* partial, int nparts, int stride, int nslots,
                            double* out, hipStream_t st);
edx_status k_coef_scale2(double* coef, const double* scale, int m, hipStream_t st);

// ---------------------------------------------------------------- tridiagonal
namespace {

// number of eigenvalues of T (diag a[0..m), off b[0..m-1)) smaller than x
int sturm_count(const double* a, const double* b, int m, double x, double tiny) {
  int cnt = 0;
  double q = a[0] - x;
  if (q < 0) ++cnt;
  for (int i = 1; i < m; ++i) {
    if (std::fabs(q) < tiny) q = -tiny;
    q = a[i] - x - b[i - 1] * b[i - 1] / q;
    if (q < 0) ++cnt;
  }
  return cnt;
}

}  // namespace

// k-th smallest eigenvalue (k = 0, 1, ...) of the symmetric tridiagonal matrix.
double tridiag_lowest(const double* a, const double* b, int m, int k) {
  if (m == 1) return a[0];
  double lo = a[0], hi = a[0], nrm = 0.0;
  for (int i = 0; i < m; ++i) {
    const double r = (i > 0 ? std::fabs(b[i - 1]) : 0.0) + (i < m - 1 ? std::fabs(b[i]) : 0.0);
    lo = std::min(lo, a[i] - r);
    hi = std::max(hi, a[i] + r);
    nrm = std::max(nrm, std::fabs(a[i]) + r);
  }
  const double tiny = std::max(nrm, 1.0) * 1e-300;
  const double eps = std::numeric_limits<double>::epsilon();
  lo -= eps * nrm + tiny;
  hi += eps * nrm + tiny;
  for (int it = 0; it < 200; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (mid <= lo || mid >= hi) break;
    if (sturm_count(a, b, m, mid, tiny) > k)
      hi = mid;
    else
      lo = mid;
    if (hi - lo <= 2.0 * eps * std::max(std::fabs(lo), std::fabs(hi))) break;
  }
  return 0.5 * (lo + hi);
}

// Eigenvector of T for eigenvalue lam by inverse iteration, Gaussian
// elimination with partial pivoting on (T - lam I).  y is normalised, with a
// positive component of largest magnitude.
void tridiag_vector(const double* a, const double* b, int m, double lam, double* y) {
  if (m == 1) {
    y[0] = 1.0;
    return;
  }
  double nrm = 0.0;
  for (int i = 0; i < m; ++i) nrm = std::max(nrm, std::fabs(a[i]) + (i < m - 1 ? std::fabs(b[i]) : 0.0));
  const double tiny = std::max(nrm, 1e-300) * std::numeric_limits<double>::epsilon();
  std::vector<double> u0(m), u1(m), u2(m), f(m), r(m);
  std::vector<int> sw(m);
  // factorisation (independent of the right-hand side)
  double c0 = a[0] - lam, c1 = m > 1 ? b[0] : 0.0, c2 = 0.0;   // candidate row k
  for (int k = 0; k < m - 1; ++k) {
    const double n0 = b[k], n1 = a[k + 1] - lam, n2 = (k + 1 < m - 1) ? b[k + 1] : 0.0;
    if (std::fabs(n0) > std::fabs(c0)) {
      sw[k] = 1;
      u0[k] = n0; u1[k] = n1; u2[k] = n2;
      const double fk = c0 / n0;
      f[k] = fk;
      c0 = c1 - fk * n1;
      c1 = c2 - fk * n2;
      c2 = 0.0;
    } else {
      sw[k] = 0;
      if (std::fabs(c0) < tiny) c0 = tiny;
      u0[k] = c0; u1[k] = c1; u2[k] = c2;
      const double fk = n0 / c0;
      f[k] = fk;
      c0 = n1 - fk * c1;
      c1 = n2 - fk * c2;
      c2 = 0.0;
    }
  }
  if (std::fabs(c0) < tiny) c0 = tiny;
  u0[m - 1] = c0; u1[m - 1] = 0.0; u2[m - 1] = 0.0;
  for (int i = 0; i < m; ++i) y[i] = 1.0;
  for (int iter = 0; iter < 3; ++iter) {
    // forward elimination of the right-hand side
    double cr = y[0];
    for (int k = 0; k < m - 1; ++k) {
      const double nr = y[k + 1];
      if (sw[k]) {
        r[k] = nr;
        cr = cr - f[k] * nr;
      } else {
        r[k] = cr;
        cr = nr - f[k] * cr;
      }
    }
    r[m - 1] = cr;
    // back substitution
    for (int k = m - 1; k >= 0; --k) {
      double s = r[k];
      if (k + 1 < m) s -= u1[k] * y[k + 1];
      if (k + 2 < m) s -= u2[k] * y[k + 2];
      y[k] = s / u0[k];
    }
    double n2 = 0.0, big = 0.0;
    int ib = 0;
    for (int i = 0; i < m; ++i) {
      n2 += y[i] * y[i];
      if (std::fabs(y[i]) > big) { big = std::fabs(y[i]); ib = i; }
    }
    const double inv = (y[ib] < 0 ? -1.0 : 1.0) / std::sqrt(n2);
    for (int i = 0; i < m; ++i) y[i] *= inv;
  }
}

// Eigenvalues and squared first components of the symmetric tridiagonal
// matrix (diagonal a[0..m), off-diagonal b[0..m-1)): the poles and weights of
// a Krylov spectral function.  Implicit symmetric QR with the Wilkinson shift
// (Golub and Van Loan, symmetric QR step): each sweep chases the bulge of one
// Givens rotation down the active block; only the first row q of the
// accumulated rotations Q (T = Q diag(theta) Q^T) is kept, so a sweep costs
// O(m) and the whole spectrum O(m^2).  Returns false if a block fails to
// converge in 60 sweeps per eigenvalue.
bool tridiag_spectrum(const double* a, const double* b, int m, double* theta, double* w) {
  if (m <= 0) return true;
  std::vector<double> d(a, a + m), e(m, 0.0), q(m, 0.0);
  for (int i = 0; i + 1 < m; ++i) e[i] = b[i];
  q[0] = 1.0;
  const double eps = std::numeric_limits<double>::epsilon();
  int h = m - 1;
  long budget = 60L * m + 60;
  while (h > 0) {
    // deflate converged off-diagonals at the bottom
    if (std::fabs(e[h - 1]) <= eps * (std::fabs(d[h - 1]) + std::fabs(d[h])) ||
        e[h - 1] == 0.0) {
      e[h - 1] = 0.0;
      --h;
      continue;
    }
    // top of the unreduced block ending at h
    int l = h - 1;
    while (l > 0 && !(std::fabs(e[l - 1]) <= eps * (std::fabs(d[l - 1]) + std::fabs(d[l])))) --l;
    if (l > 0) e[l - 1] = 0.0;
    if (--budget < 0) return false;
    // Wilkinson shift from the trailing 2x2 of the block
    const double dl = 0.5 * (d[h - 1] - d[h]);
    const double eh = e[h - 1];
    const double den = dl + (dl >= 0.0 ? 1.0 : -1.0) * std::hypot(dl, eh);
    const double mu = den != 0.0 ? d[h] - eh * eh / den : d[h];
    double x = d[l] - mu, y = e[l];
    for (int k = l; k < h; ++k) {
      const double r = std::hypot(x, y);
      const double c = r != 0.0 ? x / r : 1.0;
      const double sn = r != 0.0 ? y / r : 0.0;
      if (k > l) e[k - 1] = r;                      // the bulge at (k-1, k+1) is gone
      const double ak = d[k], bk = e[k], ck = d[k + 1];
      d[k] = c * c * ak + 2.0 * c * sn * bk + sn * sn * ck;
      d[k + 1] = sn * sn * ak - 2.0 * c * sn * bk + c * c * ck;
      e[k] = c * sn * (ck - ak) + (c * c - sn * sn) * bk;
      if (k + 1 < h) {                               // new bulge at (k, k+2)
        y = sn * e[k + 1];
        e[k + 1] = c * e[k + 1];
        x = e[k];
      }
      const double qk = q[k], qk1 = q[k + 1];
      q[k] = c * qk + sn * qk1;
      q[k + 1] = -sn * qk + c * qk1;
    }
  }
  std::vector<int> ord(m);
  for (int i = 0; i < m; ++i) ord[i] = i;
  std::sort(ord.begin(), ord.end(), [&](int x, int y) { return d[x] < d[y]; });
  for (int i = 0; i < m; ++i) {
    theta[i] = d[ord[i]];
    w[i] = q[ord[i]] * q[ord[i]];
  }
  return true;
}

// ---------------------------------------------------------------- workspace
namespace {

struct LanczosWs {
  char* vec = nullptr;       // 3 rotating vectors, or niter+1 basis vectors
  char* psi = nullptr;       // psi0 accumulator in the padded layout (or nullptr)
  size_t vstride = 0;        // bytes between vectors
  int nvec = 0;
  double* partial = nullptr; // nslots * kMaxPartials (or hv blocks)
  int partial_cap = 0;       // doubles per slot
  double* alpha = nullptr;   // [niter + 2]
  double* beta = nullptr;    // [niter + 2]   beta[j] couples j-1 and j; beta[0] = |u0|
  double* scale = nullptr;   // [niter + 2]   1/|u_j|
  double* coef = nullptr;    // [niter + 2]
  double* y = nullptr;       // [niter + 2]
  double* alpha2 = nullptr;  // replay copies
  double* beta2 = nullptr;
  double* scale2 = nullptr;
  double* gbuf = nullptr;    // Green: 2 * kMaxLmats
};

constexpr int kMaxLmats = 65536;

// vlen: elements per Krylov vector (ld * D_dw); psi_acc: reserve a vector for
// accumulating psi0 in that layout (when it differs from the dense output)
size_t lanczos_ws_layout(int64_t vlen, int vtype, int niter, int reorth, int hv_blocks,
                         bool psi_acc, char* base, LanczosWs* L) {
  const size_t vs = align_up((size_t)vlen * vbytes(vtype));
  const int nvec = reorth >= 2 ? niter + 1 : 3;   // 2 and 3 keep the basis
  const int slots = reorth == 2 ? std::max(niter + 1, 2) : 2;
  const int pcap = std::max(kMaxPartials, hv_blocks);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off += align_up(bytes);
    return base ? base + o : nullptr;
  };
  char* vec = take(vs * nvec);
  char* psi = psi_acc ? take(vs) : nullptr;
  double* partial = (double*)take(sizeof(double) * (size_t)std::max(slots * kMaxPartials, pcap));
  // (at least 8: the degeneracy check keeps scalars in coef[2..4])
  const size_t ns = sizeof(double) * (size_t)std::max(niter + 2, 8);
  double* alpha = (double*)take(ns);
  double* beta = (double*)take(ns);
  double* scale = (double*)take(ns);
  double* coef = (double*)take(ns);
  double* y = (double*)take(ns);
  double* alpha2 = (double*)take(ns);
  double* beta2 = (double*)take(ns);
  double* scale2 = (double*)take(ns);
  if (L) {
    L->vec = vec; L->psi = psi; L->vstride = vs; L->nvec = nvec; L->partial = partial;
    L->partial_cap = pcap; L->alpha = alpha; L->beta = beta; L->scale = scale;
    L->coef = coef; L->y = y; L->alpha2 = alpha2; L->beta2 = beta2; L->scale2 = scale2;
  }
  return off;
}

struct StepBufs {
  void* cur;
  void* prev;
  void* w;
};

StepBufs bufs_for(const LanczosWs& L, int j, int reorth) {
  StepBufs b;
  if (reorth >= 2) {
    b.cur = L.vec + (size_t)j * L.vstride;
    b.prev = j > 0 ? L.vec + (size_t)(j - 1) * L.vstride : nullptr;
    b.w = L.vec + (size_t)(j + 1) * L.vstride;
  } else {
    b.cur = L.vec + (size_t)(j % 3) * L.vstride;
    b.prev = j > 0 ? L.vec + (size_t)((j + 2) % 3) * L.vstride : nullptr;
    b.w = L.vec + (size_t)((j + 1) % 3) * L.vstride;
  }
  return b;
}

// One Lanczos step j: w = H v_j, alpha_j, three-term update, optional
// re-orthogonalisation, beta_{j+1} and scale_{j+1}.  psi/ycoef accumulate
// psi += y_j v_j (replay).
// defl (nullable): a unit vector x (times *defl_scale) projected out of every
// new vector, w -= <w, x> x, with the coefficient in defl_coef[0] (the
// degeneracy check of the ground state: Lanczos on the complement of psi0).
edx_status lanczos_step(const edx_sector* s, int vtype, const LanczosWs& L, int j, int reorth,
                        double* alpha, double* beta, double* scale, void* psi,
                        const double* ycoef, hipStream_t st, const char* locked = nullptr,
                        int nlock = 0, const void* defl = nullptr,
                        const double* defl_scale = nullptr, double* defl_coef = nullptr) {
  const StepBufs b = bufs_for(L, j, reorth);
  const int64_t n = s->vlen;
  const int hb = hv_partial_blocks(s, vtype);
  EDX_TRY(hv_launch(s, vtype, b.cur, b.w, s->ld, scale + j, L.partial, st));
  EDX_TRY(k_alpha_finish(L.partial, hb, alpha + j, st));
  EDX_TRY(k_update(vtype, b.w, b.cur, scale + j, b.prev, j > 0 ? scale + j - 1 : nullptr,
                   alpha + j, beta + j, n, psi, ycoef, L.partial, st));
  if (defl) {
    EDX_TRY(k_dot2(vtype, b.w, defl, defl_scale, nullptr, nullptr, n, L.partial, st));
    EDX_TRY(k_reduce_strided(L.partial, elem_blocks(n), kMaxPartials, 1, defl_coef, st));
    EDX_TRY(k_axpy2(vtype, b.w, defl, defl_coef, defl_scale, nullptr, nullptr, nullptr, n,
                    L.partial, st));
  }
  if (reorth == 1) {
    EDX_TRY(k_dot2(vtype, b.w, b.cur, scale + j, b.prev, j > 0 ? scale + j - 1 : nullptr, n,
                   L.partial, st));
    EDX_TRY(k_reduce_strided(L.partial, elem_blocks(n), kMaxPartials, 2, L.coef, st));
    EDX_TRY(k_axpy2(vtype, b.w, b.cur, L.coef, scale + j, b.prev, L.coef + 1,
                    j > 0 ? scale + j - 1 : nullptr, n, L.partial, st));
  } else if (reorth == 2) {
    const int64_t ldv = (int64_t)(L.vstride / vbytes(vtype));
    for (int pass = 0; pass < 2; ++pass) {
      if (nlock > 0) {
        // deflation: the locked (orthonormal) eigenvectors are projected out
        EDX_TRY(k_multi_dot(vtype, locked, ldv, nlock, b.w, n, L.partial, st));
        EDX_TRY(k_reduce_strided(L.partial, multi_blocks(n), kMaxPartials, nlock, L.coef, st));
        EDX_TRY(k_multi_axpy(vtype, b.w, locked, ldv, nlock, L.coef, n, L.partial, st));
      }
      EDX_TRY(k_multi_dot(vtype, L.vec, (int64_t)(L.vstride / vbytes(vtype)), j + 1, b.w, n,
                          L.partial, st));
      EDX_TRY(k_reduce_strided(L.partial, multi_blocks(n), kMaxPartials, j + 1, L.coef, st));
      EDX_TRY(k_coef_scale2(L.coef, scale, j + 1, st));
      EDX_TRY(k_multi_axpy(vtype, b.w, L.vec, (int64_t)(L.vstride / vbytes(vtype)), j + 1,
                           L.coef, n, L.partial, st));
    }
  }
  const int eb = reorth == 2 ? multi_blocks(n) : elem_blocks(n);
  EDX_TRY(k_beta_finish(L.partial, eb, beta + j + 1, scale + j + 1, st));
  return EDX_OK;
}

struct StopState {
  double tnorm = 0.0;
  double Eprev = NAN;
};

// Lowest level of H restricted to the complement of the unit vector x
// (device, Krylov layout, any positive multiple of it): plain Lanczos from a
// random start vector with x projected out of every vector.  Stops when a Ritz
// value comes within gs_threshold of e0 (degenerate), when the lowest Ritz
// value settles (tol, floored for FP32 vectors), at breakdown or after niter
// steps.  Uses the rotating vectors and the replay scalars of L.
edx_status check_degeneracy(const edx_sector* s, const edx_lanczos_opts* o, const LanczosWs& L,
                            const void* x, double e0, double tnorm, hipStream_t st, double* e1,
                            bool* degenerate) {
  const int vtype = o->vtype;
  const int niter = o->niter;
  const int64_t n = s->vlen;
  const double floor32 = vtype == EDX_F32 ? 2.0 * 1.1920929e-7 * tnorm : 0.0;
  const double thr = std::max(1e-9 * std::max(1.0, std::fabs(e0)), floor32);
  double* xs = L.coef + 3;      // 1 / |x|
  double* xc = L.coef + 4;      // projection coefficient
  EDX_TRY(k_norm2(vtype, x, n, L.partial, st));
  EDX_TRY(k_beta_finish(L.partial, elem_blocks(n), L.coef + 2, xs, st));
  // start vector orthogonal to x (another counter-based stream than the
  // ground-state run's)
  EDX_TRY(k_start_vector(vtype, L.vec, s->dup, s->ld, s->ddw * s->dph,
                         o->seed ^ 0xD1B54A32D192ED03ull, L.partial, st));
  EDX_TRY(k_dot2(vtype, L.vec, x, xs, nullptr, nullptr, n, L.partial, st));
  EDX_TRY(k_reduce_strided(L.partial, elem_blocks(n), kMaxPartials, 1, xc, st));
  EDX_TRY(k_axpy2(vtype, L.vec, x, xc, xs, nullptr, nullptr, nullptr, n, L.partial, st));
  EDX_TRY(k_beta_finish(L.partial, elem_blocks(n), L.beta2, L.scale2, st));
  double u0 = 0.0;
  EDX_HIP(hipMemcpyAsync(&u0, L.beta2, sizeof(double), hipMemcpyDeviceToHost, st));
  EDX_HIP(hipStreamSynchronize(st));
  if (!(u0 > 1e-6)) {
    // the start vector (|u| ~ sqrt(D/3) before the projection) lies in the
    // span of x: the complement is empty (D = 1) or numerically absent
    *e1 = NAN;
    *degenerate = false;
    return EDX_OK;
  }
  EDX_HIP(hipMemsetAsync(L.beta2, 0, sizeof(double), st));
  std::vector<double> ha(niter + 2), hb(niter + 2);
  const int every = std::max(1, o->check_every);
  double th = NAN, thold = NAN, tn = tnorm;
  bool deg = false;
  int done = 0;
  bool stop = false;
  while (done < niter && !stop) {
    const int upto = std::min(niter, done + every);
    for (int j = done; j < upto; ++j)
      EDX_TRY(lanczos_step(s, vtype, L, j, 0, L.alpha2, L.beta2, L.scale2, nullptr, nullptr, st,
                           nullptr, 0, x, xs, xc));
    EDX_HIP(hipMemcpyAsync(ha.data(), L.alpha2, sizeof(double) * upto, hipMemcpyDeviceToHost, st));
    EDX_HIP(hipMemcpyAsync(hb.data(), L.beta2, sizeof(double) * (upto + 1), hipMemcpyDeviceToHost,
                           st));
    EDX_HIP(hipStreamSynchronize(st));
    for (int j = done; j < upto; ++j) {
      tn = std::max(tn, std::fabs(ha[j]) + hb[j] + hb[j + 1]);
      th = tridiag_lowest(ha.data(), hb.data() + 1, j + 1, 0);
      if (th - e0 < thr) {
        deg = true;
        stop = true;
        break;
      }
      const bool bd = !(hb[j + 1] > 1e-12 * tn);
      const bool settled = j > 0 && std::fabs(th - thold) <=
                                        std::max(o->tol * std::max(1.0, std::fabs(th)), floor32);
      thold = th;
      if (bd || settled) {
        stop = true;
        break;
      }
    }
    done = upto;
  }
  *e1 = th;
  *degenerate = deg;
  return EDX_OK;
}

}  // namespace

size_t lanczos_workspace_bytes(const edx_sector* s, int vtype, int niter, int reorth) {
  return lanczos_ws_layout(s->vlen, vtype, niter, reorth, hv_partial_blocks(s, vtype),
                           s->ld != s->dup, nullptr, nullptr) + 256;
}

edx_status lanczos_ground_state_impl(const edx_sector* s, const edx_lanczos_opts* o, void* ws,
                                     size_t ws_bytes, double* e0, void* psi0,
                                     edx_lanczos_report* rep, hipStream_t st) {
  const int vtype = o->vtype;
  const int niter = o->niter;
  const int reorth = o->reorth;
  LanczosWs L;
  char* base = reinterpret_cast<char*>(align_up(reinterpret_cast<uintptr_t>(ws)));
  const size_t need = lanczos_ws_layout(s->vlen, vtype, niter, reorth,
                                        hv_partial_blocks(s, vtype), s->ld != s->dup, base, &L);
  if (need + (size_t)(base - (char*)ws) > ws_bytes) {
    set_error("lanczos: workspace too small (need " + std::to_string(need + 256) + " bytes)");
    return EDX_E_NOMEM;
  }
  const int64_t n = s->vlen;
  // start vector u_0 (random, or the caller's) and scale_0 = 1/|u_0|
  EDX_TRY(k_start_vector(vtype, L.vec, s->dup, s->ld, s->ddw * s->dph, o->seed, L.partial, st,
                         o->start));
  EDX_TRY(k_beta_finish(L.partial, elem_blocks(n), L.beta, L.scale, st));
  if (o->start) {
    double u0 = 0.0;
    EDX_HIP(hipMemcpyAsync(&u0, L.beta, sizeof(double), hipMemcpyDeviceToHost, st));
    EDX_HIP(hipStreamSynchronize(st));
    if (!(u0 > 0.0) || !std::isfinite(u0)) {
      set_error("lanczos: the start vector is zero or not finite");
      return EDX_E_INVALID;
    }
  }
  EDX_HIP(hipMemsetAsync(L.beta, 0, sizeof(double), st));   // beta_0 couples nothing

  std::vector<double> ha(niter + 2), hb(niter + 2);
  int m = 0;              // number of Lanczos steps kept (size of T)
  int done = 0;           // steps enqueued
  bool converged = false, breakdown = false;
  double E = 0.0, Eold = NAN, tnorm = 0.0, resid = 0.0;
  const int every = std::max(1, o->check_every);
  while (done < niter && m == 0) {
    const int upto = std::min(niter, done + every);
    for (int j = done; j < upto; ++j)
      EDX_TRY(lanczos_step(s, vtype, L, j, reorth, L.alpha, L.beta, L.scale, nullptr, nullptr, st));
    EDX_HIP(hipMemcpyAsync(ha.data(), L.alpha, sizeof(double) * upto, hipMemcpyDeviceToHost, st));
    EDX_HIP(hipMemcpyAsync(hb.data(), L.beta, sizeof(double) * (upto + 1), hipMemcpyDeviceToHost, st));
    EDX_HIP(hipStreamSynchronize(st));
    for (int j = done; j < upto; ++j) {
      // T_j: alpha[0..j], off-diagonal beta[1..j]
      tnorm = std::max(tnorm, std::fabs(ha[j]) + hb[j] + hb[j + 1]);
      E = tridiag_lowest(ha.data(), hb.data() + 1, j + 1, 0);
      const bool bd = !(hb[j + 1] > 1e-12 * tnorm);
      // FP32 vectors cannot resolve energies or residuals below ~eps_32 |T|:
      // the thresholds are floored there (precision mode)
      const double floor32 = vtype == EDX_F32 ? 2.0 * 1.1920929e-7 * tnorm : 0.0;
      bool ok = j > 0 &&
                std::fabs(E - Eold) <= std::max(o->tol * std::max(1.0, std::fabs(E)), floor32);
      if (ok && o->rtol > 0.0) {
        std::vector<double> yv(j + 1);
        tridiag_vector(ha.data(), hb.data() + 1, j + 1, E, yv.data());
        resid = hb[j + 1] * std::fabs(yv[j]);
        ok = resid <= std::max(o->rtol * std::max(1.0, std::fabs(E)), floor32);
      }
      Eold = E;
      if (ok || bd || j + 1 == niter) {
        m = j + 1;
        converged = ok || bd;
        breakdown = bd;
        break;
      }
    }
    done = upto;
  }
  if (m == 0) m = niter;
  E = tridiag_lowest(ha.data(), hb.data() + 1, m, 0);
  std::vector<double> y(m);
  tridiag_vector(ha.data(), hb.data() + 1, m, E, y.data());
  if (resid == 0.0) resid = hb[m] * std::fabs(y[m - 1]);
  // second Ritz value that is not a numerical copy of E (ghost copies of a
  // converged eigenvalue appear in plain Lanczos)
  double E1 = E;
  for (int k = 1; k < m; ++k) {
    const double x = tridiag_lowest(ha.data(), hb.data() + 1, m, k);
    if (x - E > 1e-10 * std::max(1.0, std::fabs(E))) { E1 = x; break; }
  }
  bool degenerate = m > 1 && E1 > E && (E1 - E) < 1e-9;

  // psi0 is accumulated in the layout of the Krylov vectors, then written
  // densely (D elements) into the caller's buffer
  void* acc = psi0 ? (L.psi ? (void*)L.psi : psi0) : nullptr;
  if (psi0) {
    if (reorth >= 2) {
      // psi0 from the stored basis (full re-orthogonalisation, or plain with
      // the basis kept)
      std::vector<double> hs(m);
      EDX_HIP(hipMemcpyAsync(hs.data(), L.scale, sizeof(double) * m, hipMemcpyDeviceToHost, st));
      EDX_HIP(hipStreamSynchronize(st));
      std::vector<double> c(m);
      for (int k = 0; k < m; ++k) c[k] = -y[k] * hs[k];
      EDX_HIP(hipMemcpyAsync(L.coef, c.data(), sizeof(double) * m, hipMemcpyHostToDevice, st));
      EDX_HIP(hipMemsetAsync(acc, 0, (size_t)n * vbytes(vtype), st));
      EDX_TRY(k_multi_axpy(vtype, acc, L.vec, (int64_t)(L.vstride / vbytes(vtype)), m, L.coef, n,
                           nullptr, st));
    } else {
      // replay: identical start vector and recurrence, psi += y_j v_j
      EDX_HIP(hipMemcpyAsync(L.y, y.data(), sizeof(double) * m, hipMemcpyHostToDevice, st));
      EDX_HIP(hipMemsetAsync(acc, 0, (size_t)n * vbytes(vtype), st));
      EDX_TRY(k_start_vector(vtype, L.vec, s->dup, s->ld, s->ddw * s->dph, o->seed, L.partial, st,
                             o->start));
      EDX_TRY(k_beta_finish(L.partial, elem_blocks(n), L.beta2, L.scale2, st));
      EDX_HIP(hipMemsetAsync(L.beta2, 0, sizeof(double), st));
      for (int j = 0; j < m; ++j)
        EDX_TRY(lanczos_step(s, vtype, L, j, reorth, L.alpha2, L.beta2, L.scale2, acc, L.y + j,
                             st));
    }
    // normalise psi0
    EDX_TRY(k_norm2(vtype, acc, n, L.partial, st));
    EDX_TRY(k_beta_finish(L.partial, elem_blocks(n), L.coef, L.coef + 1, st));
    if (L.psi)
      EDX_TRY(k_unpad_scale(vtype, acc, s->ld, s->dup, s->ddw * s->dph, L.coef + 1, psi0, st));
    else
      EDX_TRY(k_scale_copy(vtype, psi0, L.coef + 1, psi0, n, st));
    EDX_HIP(hipStreamSynchronize(st));
  }
  if (acc && o->degen_check && converged) {
    // A run from one start vector holds one vector of a degenerate level, so
    // a second plain run is kept orthogonal to psi0 (projected out of the
    // start vector and of every new vector).  Its Ritz values bound the
    // lowest level of the complement from above: one within gs_threshold of
    // E0 means a degenerate ground level; otherwise the run goes on until its
    // lowest Ritz value settles (that is E1).
    double E1d = NAN;
    EDX_TRY(check_degeneracy(s, o, L, acc, E, tnorm, st, &E1d, &degenerate));
    E1 = E1d;
  }
  *e0 = E;
  if (rep) {
    rep->iters = m;
    rep->converged = converged ? 1 : 0;
    rep->breakdown = breakdown ? 1 : 0;
    rep->degenerate = degenerate ? 1 : 0;
    rep->e0 = E;
    rep->e1 = E1;
    rep->beta_last = hb[m];
    rep->resid = resid;
  }
  if (!converged) {
    set_error("lanczos: stop rule not met within niter");
    return EDX_E_NOCONV;
  }
  if (degenerate) return EDX_E_DEGENERATE;
  return EDX_OK;
}

// ---------------------------------------------------------------- low-lying states
// Workspace: the Lanczos basis of one run (full re-orthogonalisation) and k + 2
// vectors after it: k locked eigenvectors (orthonormal, padded layout), one
// staging slot for a Ritz vector that is not locked yet and one for H x when a
// candidate's residual is checked.
namespace {

size_t lowest_ws_layout(int64_t vlen, int vtype, int niter, int k, int hvb, char* base,
                        LanczosWs* L, char** locked) {
  const int nit = std::max(niter, k + 1);   // scalar arrays and dot slots cover k
  const size_t off = lanczos_ws_layout(vlen, vtype, nit, 2, hvb, false, base, L);
  if (locked) *locked = base ? base + off : nullptr;
  // k locked vectors, a staging slot and a residual slot
  return off + align_up((size_t)vlen * vbytes(vtype)) * (size_t)(k + 2);
}

// y -= sum_q <Y_q, y> Y_q over orthonormal Y_q (two passes), then normalise;
// false if y lies (to 1e-8 of its norm) in their span or is not finite
bool orthonormalise_against(const std::vector<std::vector<double>>& Y, std::vector<double>& y) {
  const size_t m = y.size();
  double n0 = 0.0;
  for (double x : y) n0 += x * x;
  n0 = std::sqrt(n0);
  if (!(n0 > 0.0) || !std::isfinite(n0)) return false;
  for (int pass = 0; pass < 2; ++pass)
    for (const std::vector<double>& q : Y) {
      double d = 0.0;
      for (size_t j = 0; j < m; ++j) d += q[j] * y[j];
      for (size_t j = 0; j < m; ++j) y[j] -= d * q[j];
    }
  double nn = 0.0;
  for (double x : y) nn += x * x;
  nn = std::sqrt(nn);
  if (!(nn > 1e-8 * n0)) return false;
  for (double& x : y) x /= nn;
  return true;
}

// Thick restart.  Keeping l orthonormal Ritz vectors x = V Y of a run that hit
// niter gives H x = x G + v_m s^T with G = Y^T T Y (l x l) and s = beta_m Y[m-1, :];
// with v_m appended the projected matrix is the arrow [[G, s], [s^T, .]].
// Householder reflections on the first l indices, taken from the last row up,
// bring it back to tridiagonal form without moving v_m, so the recurrence
// continues from step l as a plain Lanczos run would.  A is (l+1) x (l+1),
// row-major; on return a[0..l) is the diagonal, b[1..l] the couplings (b[i]
// between i-1 and i, b[l] between l-1 and v_m), all >= 0, and Q (l x l,
// row-major) the change of basis of the kept vectors.
void arrow_to_tridiag(std::vector<double> A, int l, double* a, double* b,
                      std::vector<double>& Q) {
  const int n = l + 1;
  Q.assign((size_t)l * l, 0.0);
  for (int i = 0; i < l; ++i) Q[(size_t)i * l + i] = 1.0;
  auto at = [&](int i, int j) -> double& { return A[(size_t)i * n + j]; };
  std::vector<double> u(n);
  for (int r = l; r >= 2; --r) {
    // reflect x = A[r, 0..r) onto a multiple of e_{r-1}
    double low = 0.0, nrm = 0.0;
    for (int k = 0; k < r; ++k) {
      nrm += at(r, k) * at(r, k);
      if (k < r - 1) low += at(r, k) * at(r, k);
    }
    if (low == 0.0) continue;
    nrm = std::sqrt(nrm);
    const double al = at(r, r - 1) >= 0.0 ? -nrm : nrm;
    double un = 0.0;
    for (int k = 0; k < r; ++k) {
      u[k] = at(r, k) - (k == r - 1 ? al : 0.0);
      un += u[k] * u[k];
    }
    un = std::sqrt(un);
    for (int k = 0; k < r; ++k) u[k] /= un;
    for (int c = 0; c < n; ++c) {            // A <- P A
      double t = 0.0;
      for (int k = 0; k < r; ++k) t += u[k] * at(k, c);
      for (int k = 0; k < r; ++k) at(k, c) -= 2.0 * u[k] * t;
    }
    for (int i = 0; i < n; ++i) {            // A <- A P
      double t = 0.0;
      for (int k = 0; k < r; ++k) t += at(i, k) * u[k];
      for (int k = 0; k < r; ++k) at(i, k) -= 2.0 * t * u[k];
    }
    for (int i = 0; i < l; ++i) {            // Q <- Q P
      double t = 0.0;
      for (int k = 0; k < r; ++k) t += Q[(size_t)i * l + k] * u[k];
      for (int k = 0; k < r; ++k) Q[(size_t)i * l + k] -= 2.0 * t * u[k];
    }
  }
  for (int i = 0; i < l; ++i) a[i] = at(i, i);
  for (int i = 1; i <= l; ++i) b[i] = at(i, i - 1);
  // signs: flip kept vectors so every coupling is >= 0 (v_m keeps its sign)
  std::vector<double> d(n, 1.0);
  for (int i = l; i >= 1; --i) d[i - 1] = b[i] * d[i] < 0.0 ? -1.0 : 1.0;
  for (int i = 1; i <= l; ++i) b[i] = std::fabs(b[i]);
  for (int i = 0; i < l; ++i)
    for (int c = 0; c < l; ++c) Q[(size_t)i * l + c] *= d[c];
}

// w -= sum_k <x_k, w> x_k over nl orthonormal x_k, twice; L.partial then holds
// the partial sums of |w|^2 (multi_blocks(n) of them)
edx_status project_out(int vtype, void* w, const char* X, const LanczosWs& L, int nl, int64_t n,
                       hipStream_t st) {
  const int64_t ldv = (int64_t)(L.vstride / vbytes(vtype));
  for (int pass = 0; pass < 2; ++pass) {
    EDX_TRY(k_multi_dot(vtype, X, ldv, nl, w, n, L.partial, st));
    EDX_TRY(k_reduce_strided(L.partial, multi_blocks(n), kMaxPartials, nl, L.coef, st));
    EDX_TRY(k_multi_axpy(vtype, w, X, ldv, nl, L.coef, n, L.partial, st));
  }
  return EDX_OK;
}

// out = sum_i c_i sum_j y_i[j] v_j over the run's basis (v_j = scale_j u_j)
edx_status ritz_combination(int vtype, const LanczosWs& L, int m, const std::vector<double>& hs,
                            const std::vector<std::vector<double>>& ys,
                            const std::vector<double>& c, void* out, int64_t n, hipStream_t st) {
  std::vector<double> coef(m, 0.0);
  for (size_t i = 0; i < ys.size(); ++i)
    for (int j = 0; j < m; ++j) coef[j] -= c[i] * ys[i][j] * hs[j];
  EDX_HIP(hipMemcpyAsync(L.coef, coef.data(), sizeof(double) * m, hipMemcpyHostToDevice, st));
  EDX_HIP(hipMemsetAsync(out, 0, (size_t)n * vbytes(vtype), st));
  EDX_TRY(k_multi_axpy(vtype, out, L.vec, (int64_t)(L.vstride / vbytes(vtype)), m, L.coef, n,
                       nullptr, st));
  EDX_HIP(hipStreamSynchronize(st));   // coef is a host temporary
  return EDX_OK;
}

constexpr int kMaxRestarts = 64;   // thick restarts per run

// Thick restart of a run whose basis holds mm vectors: the lowest lk Ritz
// vectors become basis vectors 0..lk-1, v_mm becomes vector lk, and alpha,
// beta, scale (device) and ha, hb (host) describe the tridiagonal of the new
// basis (arrow_to_tridiag), so the next step is j = lk.
edx_status thick_restart(const edx_sector* s, int vtype, const LanczosWs& L, int mm, int& lk,
                         std::vector<double>& ha, std::vector<double>& hb, hipStream_t st) {
  const int64_t n = s->vlen;
  const int64_t ldv = (int64_t)(L.vstride / vbytes(vtype));
  // Ritz coefficient vectors, orthonormalised.  Equal or clustered Ritz values
  // (a tridiagonal that has split into blocks) give parallel inverse-iteration
  // vectors: such a vector adds no direction and is dropped, so lk may shrink
  // (lk = 0: no restart possible)
  std::vector<std::vector<double>> Y;
  for (int i = 0; i < lk; ++i) {
    std::vector<double> y(mm);
    const double th = tridiag_lowest(ha.data(), hb.data() + 1, mm, i);
    tridiag_vector(ha.data(), hb.data() + 1, mm, th, y.data());
    if (!orthonormalise_against(Y, y)) continue;
    Y.push_back(std::move(y));
  }
  lk = (int)Y.size();
  if (lk == 0) return EDX_OK;
  // arrow matrix: G = Y^T T Y and s = beta_mm Y[mm-1, :]
  std::vector<double> A((size_t)(lk + 1) * (lk + 1), 0.0), TY(mm);
  for (int c = 0; c < lk; ++c) {
    const std::vector<double>& y = Y[c];
    for (int j = 0; j < mm; ++j) {
      double t = ha[j] * y[j];
      if (j > 0) t += hb[j] * y[j - 1];
      if (j + 1 < mm) t += hb[j + 1] * y[j + 1];
      TY[j] = t;
    }
    for (int r = 0; r < lk; ++r) {
      double g = 0.0;
      for (int j = 0; j < mm; ++j) g += Y[r][j] * TY[j];
      A[(size_t)r * (lk + 1) + c] = g;
    }
    A[(size_t)lk * (lk + 1) + c] = A[(size_t)c * (lk + 1) + lk] = hb[mm] * y[mm - 1];
  }
  for (int r = 0; r < lk; ++r)        // symmetrise the rounding
    for (int c = 0; c < r; ++c) {
      const double g = 0.5 * (A[(size_t)r * (lk + 1) + c] + A[(size_t)c * (lk + 1) + r]);
      A[(size_t)r * (lk + 1) + c] = A[(size_t)c * (lk + 1) + r] = g;
    }
  std::vector<double> na(lk), nb(lk + 1), Q;
  arrow_to_tridiag(A, lk, na.data(), nb.data(), Q);
  for (int i = 0; i < lk; ++i)
    if (!std::isfinite(na[i]) || !std::isfinite(nb[i + 1])) {
      lk = 0;   // leave the basis as it is
      return EDX_OK;
    }
  // C[j][c] = scale_j sum_i Y_i[j] Q[i][c]: the stored u_j are unnormalised
  std::vector<double> hs(mm + 1);
  EDX_HIP(hipMemcpyAsync(hs.data(), L.scale, sizeof(double) * (mm + 1), hipMemcpyDeviceToHost,
                         st));
  EDX_HIP(hipStreamSynchronize(st));
  std::vector<double> C((size_t)mm * lk, 0.0);
  for (int j = 0; j < mm; ++j)
    for (int c = 0; c < lk; ++c) {
      double t = 0.0;
      for (int i = 0; i < lk; ++i) t += Y[i][j] * Q[(size_t)i * lk + c];
      C[(size_t)j * lk + c] = hs[j] * t;
    }
  EDX_HIP(hipMemcpyAsync(L.partial, C.data(), sizeof(double) * C.size(), hipMemcpyHostToDevice,
                         st));
  EDX_TRY(k_basis_rotate(vtype, L.vec, ldv, mm, lk, L.partial, n, st));
  EDX_HIP(hipMemcpyAsync(L.vec + (size_t)lk * L.vstride, L.vec + (size_t)mm * L.vstride,
                         (size_t)n * vbytes(vtype), hipMemcpyDeviceToDevice, st));
  std::vector<double> sc(lk + 1, 1.0), be(lk + 1, 0.0);
  sc[lk] = hs[mm];
  for (int i = 1; i <= lk; ++i) be[i] = nb[i];
  EDX_HIP(hipMemcpyAsync(L.scale, sc.data(), sizeof(double) * (lk + 1), hipMemcpyHostToDevice, st));
  EDX_HIP(hipMemcpyAsync(L.alpha, na.data(), sizeof(double) * lk, hipMemcpyHostToDevice, st));
  EDX_HIP(hipMemcpyAsync(L.beta, be.data(), sizeof(double) * (lk + 1), hipMemcpyHostToDevice, st));
  EDX_HIP(hipStreamSynchronize(st));   // the sources are host temporaries
  for (int i = 0; i < lk; ++i) ha[i] = na[i];
  for (int i = 0; i <= lk; ++i) hb[i] = be[i];
  return EDX_OK;
}

}  // namespace

size_t lowest_workspace_bytes(const edx_sector* s, int vtype, int niter, int k) {
  k = (int)std::min<int64_t>(std::max(k, 1), s->dim);
  return lowest_ws_layout(s->vlen, vtype, niter, k, hv_partial_blocks(s, vtype), nullptr, nullptr,
                          nullptr) + 256;
}

edx_status lowest_states_impl(const edx_sector* s, int k, const edx_lanczos_opts* o, int verify,
                              void* ws, size_t ws_bytes, double* e_out, void* psi_out,
                              edx_lowest_report* rep, hipStream_t st) {
  const int vtype = o->vtype;
  const int niter = o->niter;
  k = (int)std::min<int64_t>(k, s->dim);
  LanczosWs L;
  char* X = nullptr;
  char* base = reinterpret_cast<char*>(align_up(reinterpret_cast<uintptr_t>(ws)));
  const size_t need = lowest_ws_layout(s->vlen, vtype, niter, k, hv_partial_blocks(s, vtype),
                                       base, &L, &X);
  if (need + (size_t)(base - (char*)ws) > ws_bytes) {
    set_error("lanczos_lowest: workspace too small (need " + std::to_string(need + 256) +
              " bytes)");
    return EDX_E_NOMEM;
  }
  const int64_t n = s->vlen;
  const size_t vs = L.vstride;
  const double rtol = o->rtol > 0.0 ? o->rtol : o->tol;
  std::vector<double> E;            // energies of the locked states, slot order
  std::vector<double> ha(niter + 2), hb(niter + 2), hs(niter + 2);
  bool from_staging = false;        // next run starts from the staging slot
  bool verified = verify == 0;
  int runs = 0, iters = 0;
  double resid_max = 0.0;
  const int max_runs = 4 * k + 8;
  int stall = 0;                    // consecutive runs that locked nothing
  auto slot = [&](int i) { return X + (size_t)i * vs; };

  while (runs < max_runs) {
    const int nl = (int)E.size();
    const bool checking = nl >= k;
    if (checking && (verified || nl >= s->dim)) {
      verified = true;
      break;
    }
    // states aimed at in this run: all that remain when the run may be long,
    // fewer when niter bounds it (a short Krylov space converges only its
    // lowest few Ritz pairs; the restart then keeps their vectors)
    const int want = checking ? 1 : std::min(k - nl, std::max(1, niter / 4));
    char* stage = slot(nl);         // first free slot (slot k while checking)
    // start vector, orthogonal to the locked states
    if (from_staging) {
      EDX_HIP(hipMemcpyAsync(L.vec, stage, (size_t)n * vbytes(vtype), hipMemcpyDeviceToDevice,
                             st));
      if (nl == 0) EDX_TRY(k_norm2(vtype, L.vec, n, L.partial, st));
    } else {
      EDX_TRY(k_start_vector(vtype, L.vec, s->dup, s->ld, s->ddw * s->dph,
                             o->seed + 0x9E3779B97F4A7C15ull * (uint64_t)runs, L.partial, st));
    }
    if (nl > 0) EDX_TRY(project_out(vtype, L.vec, X, L, nl, n, st));
    // the norm's partial sums come from project_out's last kernel or from the
    // start / norm kernel: their counts differ
    EDX_TRY(k_beta_finish(L.partial, nl > 0 ? multi_blocks(n) : elem_blocks(n), L.beta, L.scale,
                          st));
    if (from_staging) {
      // a staged (unit) Ritz vector that lies in the locked span leaves almost
      // nothing after the projection: start from a random vector instead
      double b0 = 0.0;
      EDX_HIP(hipMemcpyAsync(&b0, L.beta, sizeof(double), hipMemcpyDeviceToHost, st));
      EDX_HIP(hipStreamSynchronize(st));
      if (!(b0 > 1e-6)) {
        EDX_TRY(k_start_vector(vtype, L.vec, s->dup, s->ld, s->ddw * s->dph,
                               o->seed + 0x9E3779B97F4A7C15ull * (uint64_t)runs, L.partial, st));
        if (nl > 0) EDX_TRY(project_out(vtype, L.vec, X, L, nl, n, st));
        EDX_TRY(k_beta_finish(L.partial, nl > 0 ? multi_blocks(n) : elem_blocks(n), L.beta,
                              L.scale, st));
      }
    }
    EDX_HIP(hipMemsetAsync(L.beta, 0, sizeof(double), st));
    ++runs;

    // Lanczos run with full re-orthogonalisation and deflation
    int m = 0, done = 0, done_run = 0, restarts = 0;
    double tnorm = 0.0;
    std::vector<double> theta;
    std::vector<std::vector<double>> ys;
    std::vector<double> res;
    int nconv = 0;
    const int every = std::max(1, o->check_every);
    while (done < niter && m == 0) {
      const int upto = (int)std::min<int64_t>({(int64_t)niter, (int64_t)done + every,
                                               s->dim - nl});
      for (int j = done; j < upto; ++j)
        EDX_TRY(lanczos_step(s, vtype, L, j, 2, L.alpha, L.beta, L.scale, nullptr, nullptr, st,
                             X, nl));
      EDX_HIP(hipMemcpyAsync(ha.data(), L.alpha, sizeof(double) * upto, hipMemcpyDeviceToHost,
                             st));
      EDX_HIP(hipMemcpyAsync(hb.data(), L.beta, sizeof(double) * (upto + 1),
                             hipMemcpyDeviceToHost, st));
      EDX_HIP(hipStreamSynchronize(st));
      // the first breakdown ends the run: its Krylov space is invariant (every
      // Ritz pair exact) and the vectors after it would come from rounding noise
      int mm = upto;
      bool bd = false;
      for (int j = done; j < upto; ++j) {
        tnorm = std::max(tnorm, std::fabs(ha[j]) + hb[j] + hb[j + 1]);
        if (!(hb[j + 1] > 1e-12 * tnorm)) {
          mm = j + 1;
          bd = true;
          break;
        }
      }
      bd = bd || mm >= s->dim - nl;
      const double floor32 = vtype == EDX_F32 ? 2.0 * 1.1920929e-7 * tnorm : 0.0;
      const int w = std::min(want, mm);
      theta.assign(w, 0.0);
      ys.assign(w, std::vector<double>(mm));
      res.assign(w, 0.0);
      nconv = 0;
      bool lead = true;
      for (int i = 0; i < w; ++i) {
        theta[i] = tridiag_lowest(ha.data(), hb.data() + 1, mm, i);
        tridiag_vector(ha.data(), hb.data() + 1, mm, theta[i], ys[i].data());
        res[i] = bd ? 0.0 : hb[mm] * std::fabs(ys[i][mm - 1]);
        const bool ok = res[i] <= std::max(rtol * std::max(1.0, std::fabs(theta[i])), floor32);
        lead = lead && ok;
        if (lead) ++nconv;
      }
      if (nconv == want || bd) {
        m = mm;
      } else if (upto == niter) {
        // the basis is full: thick restart with the lowest lk Ritz vectors
        int lk = std::min({std::max(want + 4, niter / 3), niter / 2, kMaxKeep, mm - 1});
        if (restarts < kMaxRestarts && lk >= 1)
          EDX_TRY(thick_restart(s, vtype, L, mm, lk, ha, hb, st));
        else
          lk = 0;
        if (lk < 1) {
          m = mm;   // no restart: the run ends here
        } else {
          ++restarts;
          iters += mm - done_run;
          done_run = lk;
          done = lk;
          continue;
        }
      }
      done = upto;
    }
    iters += m - done_run;
    // orthonormalise the Ritz coefficient vectors: a tight cluster of Ritz
    // values can give nearly parallel inverse-iteration vectors; one that adds
    // no direction is not locked (a later run finds that state)
    std::vector<char> usable(ys.size(), 1);
    {
      std::vector<std::vector<double>> done_y;
      for (size_t i = 0; i < ys.size(); ++i) {
        ys[i].resize(m);
        if (orthonormalise_against(done_y, ys[i]))
          done_y.push_back(ys[i]);
        else
          usable[i] = 0;
      }
    }
    EDX_HIP(hipMemcpyAsync(hs.data(), L.scale, sizeof(double) * m, hipMemcpyDeviceToHost, st));
    EDX_HIP(hipStreamSynchronize(st));

    // lock the converged leading pairs (or, while checking, test the lowest)
    int locked_now = 0;
    std::vector<char> took(ys.size(), 0);
    for (int i = 0; i < nconv; ++i) {
      if (!usable[i]) continue;
      if (checking) {
        const double emax = *std::max_element(E.begin(), E.end());
        const double delta = std::max(10.0 * rtol * std::max(1.0, std::fabs(emax)), 1e-12) +
                             (vtype == EDX_F32 ? 4.0 * 1.1920929e-7 * tnorm : 0.0);
        if (theta[0] >= emax - delta) {
          verified = true;
          break;
        }
      }
      char* dst = slot((int)E.size());
      EDX_TRY(ritz_combination(vtype, L, m, hs, {ys[i]}, {1.0}, dst, n, st));
      if (!E.empty()) {
        EDX_TRY(project_out(vtype, dst, X, L, (int)E.size(), n, st));
      } else {
        EDX_TRY(k_norm2(vtype, dst, n, L.partial, st));
      }
      EDX_TRY(k_beta_finish(L.partial, !E.empty() ? multi_blocks(n) : elem_blocks(n), L.coef,
                            L.coef + 1, st));
      double nrm = 0.0;
      EDX_HIP(hipMemcpyAsync(&nrm, L.coef, sizeof(double), hipMemcpyDeviceToHost, st));
      EDX_HIP(hipStreamSynchronize(st));
      if (!(nrm > 0.5)) continue;   // not independent of the locked states: leave it
      EDX_TRY(k_scale_copy(vtype, dst, L.coef + 1, dst, n, st));
      // the candidate's true residual |H x - theta x|: a Krylov space run past an
      // exhausted invariant subspace (degenerate spectrum) can produce Ritz
      // pairs whose estimate is small but whose vectors are not eigenvectors
      {
        char* tmp = slot(k + 1);
        EDX_TRY(hv_launch(s, vtype, dst, tmp, s->ld, nullptr, nullptr, st));
        const double sc[2] = {1.0, theta[i]};
        EDX_HIP(hipMemcpyAsync(L.y, sc, sizeof(sc), hipMemcpyHostToDevice, st));
        EDX_TRY(k_update(vtype, tmp, dst, L.y, nullptr, nullptr, L.y + 1, L.y + 1, n, nullptr,
                         nullptr, L.partial, st));
        EDX_TRY(k_beta_finish(L.partial, elem_blocks(n), L.alpha2, L.scale2, st));
        double rn = 0.0;
        EDX_HIP(hipMemcpyAsync(&rn, L.alpha2, sizeof(double), hipMemcpyDeviceToHost, st));
        EDX_HIP(hipStreamSynchronize(st));
        const double thr = std::max(100.0 * rtol * std::max(1.0, std::fabs(theta[i])),
                                    (vtype == EDX_F32 ? 1e-5 : 1e-9) * std::max(1.0, tnorm));
        if (!(rn <= thr)) continue;
        res[i] = std::max(res[i], rn);
      }
      if (checking) {
        // replaces the highest locked state
        const int hi = (int)(std::max_element(E.begin(), E.end()) - E.begin());
        EDX_HIP(hipMemcpyAsync(slot(hi), dst, (size_t)n * vbytes(vtype), hipMemcpyDeviceToDevice,
                               st));
        E[hi] = theta[i];
      } else {
        E.push_back(theta[i]);
      }
      resid_max = std::max(resid_max, res[i]);
      ++locked_now;
      took[i] = 1;
      if (checking) break;
    }
    if (verified && checking) break;
    // a run that locked nothing continues from its wanted Ritz vectors if it
    // reached niter (the restart), else from a fresh random vector; many runs
    // in a row without progress end the search
    stall = locked_now == 0 ? stall + 1 : 0;
    from_staging = false;
    const bool hit_niter = m >= niter;
    if (stall >= 16) break;
    const int wl = (int)ys.size();
    if ((locked_now > 0 || hit_niter) && locked_now < wl && (int)E.size() < s->dim) {
      // the lowest wanted Ritz vector not locked: a restarted single-vector
      // Lanczos keeps converging it (a sum of several would dilute it)
      std::vector<std::vector<double>> rest;
      for (int i = 0; i < wl && rest.empty(); ++i)
        if (!took[i] && usable[i]) rest.push_back(ys[i]);
      if (!rest.empty()) {
        const int free_slot = std::min((int)E.size(), k);
        EDX_TRY(ritz_combination(vtype, L, m, hs, rest, std::vector<double>(rest.size(), 1.0),
                                 slot(free_slot), n, st));
        from_staging = true;
      }
    }
  }
  const int nf = (int)E.size();
  std::vector<int> order(nf);
  for (int i = 0; i < nf; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return E[x] < E[y]; });
  for (int i = 0; i < nf; ++i) e_out[i] = E[order[i]];
  if (psi_out && nf > 0) {
    const double one = 1.0;
    EDX_HIP(hipMemcpyAsync(L.coef + 2, &one, sizeof(double), hipMemcpyHostToDevice, st));
    for (int i = 0; i < nf; ++i) {
      char* dst = reinterpret_cast<char*>(psi_out) + (size_t)i * s->dim * vbytes(vtype);
      EDX_TRY(k_unpad_scale(vtype, slot(order[i]), s->ld, s->dup, s->ddw * s->dph, L.coef + 2, dst, st));
    }
  }
  EDX_HIP(hipStreamSynchronize(st));
  if (rep) {
    rep->nfound = nf;
    rep->runs = runs;
    rep->iters = iters;
    rep->verified = verified ? 1 : 0;
    rep->resid_max = resid_max;
  }
  if (nf < k || !verified) {
    set_error("lanczos_lowest: " + std::to_string(nf) + " of " + std::to_string(k) +
              " states converged" + (verified ? "" : " (check run not passed)"));
    return EDX_E_NOCONV;
  }
  return EDX_OK;
}

// ---------------------------------------------------------------- Green
size_t green_workspace_bytes(const edx_sector* s, int vtype, int ngf) {
  // the largest neighbour sector of either spin bounds the vectors
  int64_t dmax = 1;
  const int ns = s->model.ns;
  auto comb = [](int nn, int k) -> int64_t {
    if (k < 0 || k > nn) return 0;
    int64_t r = 1;
    for (int i = 1; i <= k; ++i) r = r * (nn - k + i) / i;
    return r;
  };
  // Krylov vectors of a neighbour sector use its padded column stride (times
  // the phonon copies)
  const int64_t cu = comb(ns, s->nup), cd = comb(ns, s->ndw);
  for (int d : {-1, 1}) {
    dmax = std::max(dmax, vec_ld(comb(ns, s->nup + d)) * cd * s->dph);
    dmax = std::max(dmax, vec_ld(cu) * comb(ns, s->ndw + d) * s->dph);
  }
  // hv partial blocks of a neighbour sector: bounded by its column count per
  // phonon slice, plus the phonon pass (8 columns per workgroup and slice)
  const int64_t ddw_max = std::max({comb(ns, s->ndw - 1), comb(ns, s->ndw), comb(ns, s->ndw + 1)});
  const int hvb = (int)std::max<int64_t>(
      kMaxPartials, s->dph * (ddw_max + 8 + kNdMaxBlocks + (s->dph > 1 ? ddw_max / 8 + 1 : 0)));
  return lanczos_ws_layout(dmax, vtype, ngf, 0, hvb, false, nullptr, nullptr) +
         sizeof(double) * (2 * kMaxLmats + 4 * (ngf + 1)) + 512;
}

namespace {

// Sectors reached by d+_{orb,spin} (k = 0) and d_{orb,spin} (k = 1): total
// counts N_spin +- 1, or, in an orbital-resolved sector, orbital orb's count of
// that spin +- 1 (the other orbitals' counts are untouched).
edx_sector* const* neighbour_slot(const edx_sector* gs, int orb, int spin) {
  return gs->orb ? gs->nb_orb[spin][orb] : gs->nb[spin];
}

edx_status ensure_neighbours(const edx_sector* gs, int orb, int spin, hipStream_t st) {
  edx_sector* g = const_cast<edx_sector*>(gs);
  std::lock_guard<std::mutex> lk(g->nb_mu);
  edx_sector** slot = g->orb ? g->nb_orb[spin][orb] : g->nb[spin];
  const Allocator* alloc = gs->alloc.alloc ? &gs->alloc : nullptr;
  for (int k = 0; k < 2; ++k) {
    const int d = k == 0 ? 1 : -1;
    if (slot[k]) continue;
    edx_sector* t = nullptr;
    if (gs->orb) {
      int cu[kMaxNorb], cd[kMaxNorb];
      for (int a = 0; a < kMaxNorb; ++a) {
        cu[a] = gs->up.counts[a];
        cd[a] = gs->dw.counts[a];
      }
      int* c = spin == 0 ? cu : cd;
      c[orb] += d;
      if (c[orb] < 0 || c[orb] > gs->model.nbath + 1) continue;
      EDX_TRY(build_sector_impl(gs->model, gs->nup + (spin == 0 ? d : 0),
                                gs->ndw + (spin == 1 ? d : 0), st, &t, alloc, cu, cd));
    } else {
      const int nn = (spin == 0 ? gs->nup : gs->ndw) + d;
      if (nn < 0 || nn > gs->model.ns) continue;
      EDX_TRY(build_sector_impl(gs->model, spin == 0 ? nn : gs->nup, spin == 0 ? gs->ndw : nn,
                                st, &t, alloc));
    }
    slot[k] = t;
  }
  return EDX_OK;
}

}  // namespace

edx_status green_cf_impl(const edx_sector* gs, const void* psi0, double e0, int orb, int spin,
                         const edx_gf_opts* o, void* ws, size_t ws_bytes, double* g_host,
                         edx_gf_report* rep, hipStream_t st) {
  const int vtype = o->vtype;
  const int ngf = o->ngf;
  if (o->lmats < 1 || o->lmats > kMaxLmats || ngf < 1 || !(o->beta > 0.0)) {
    set_error("green: need 1 <= lmats <= 65536, ngf >= 1, beta > 0");
    return EDX_E_INVALID;
  }
  const size_t need = green_workspace_bytes(gs, vtype, ngf);
  if (need > ws_bytes) {
    set_error("green: workspace too small (need " + std::to_string(need) + " bytes)");
    return EDX_E_NOMEM;
  }
  EDX_TRY(ensure_neighbours(gs, orb, spin, st));
  edx_sector* const* nbs = neighbour_slot(gs, orb, spin);
  char* base = reinterpret_cast<char*>(align_up(reinterpret_cast<uintptr_t>(ws)));
  double* gdev = nullptr;
  double w[2] = {0.0, 0.0};
  int nlen[2] = {0, 0};
  std::vector<double> ha[2], hb[2];
  // the two branches run one after the other in the same workspace
  for (int br = 0; br < 2; ++br) {
    const edx_sector* t = nbs[br];
    LanczosWs L;
    lanczos_ws_layout(t ? t->vlen : 1, vtype, ngf, 0, t ? hv_partial_blocks(t, vtype) : 1, false,
                      base, &L);
    if (!t) continue;
    EDX_TRY(k_apply_op(gs, t, vtype, psi0, L.vec, orb, spin, br == 0 ? 1 : 0, st));
    EDX_TRY(k_norm2(vtype, L.vec, t->vlen, L.partial, st));
    EDX_TRY(k_beta_finish(L.partial, elem_blocks(t->vlen), L.beta, L.scale, st));
    double nrm = 0.0;
    EDX_HIP(hipMemcpyAsync(&nrm, L.beta, sizeof(double), hipMemcpyDeviceToHost, st));
    EDX_HIP(hipStreamSynchronize(st));
    w[br] = nrm * nrm;
    if (!(nrm > 0.0)) continue;
    EDX_HIP(hipMemsetAsync(L.beta, 0, sizeof(double), st));
    for (int j = 0; j < ngf; ++j)
      EDX_TRY(lanczos_step(t, vtype, L, j, 0, L.alpha, L.beta, L.scale, nullptr, nullptr, st));
    ha[br].resize(ngf + 1);
    hb[br].resize(ngf + 1);
    EDX_HIP(hipMemcpyAsync(ha[br].data(), L.alpha, sizeof(double) * ngf, hipMemcpyDeviceToHost, st));
    EDX_HIP(hipMemcpyAsync(hb[br].data(), L.beta, sizeof(double) * (ngf + 1), hipMemcpyDeviceToHost,
                           st));
    EDX_HIP(hipStreamSynchronize(st));
    // truncate at the first breakdown
    double tn = 0.0;
    int len = ngf;
    for (int j = 0; j < ngf; ++j) {
      tn = std::max(tn, std::fabs(ha[br][j]) + hb[br][j] + hb[br][j + 1]);
      if (j + 1 < ngf && !(hb[br][j + 1] > 1e-12 * tn)) {
        len = j + 1;
        break;
      }
    }
    nlen[br] = len;
  }
  // G and the staged coefficients sit after the larger of the two layouts
  size_t off = 0;
  for (int br = 0; br < 2; ++br) {
    const edx_sector* t = nbs[br];
    off = std::max(off, lanczos_ws_layout(t ? t->vlen : 1, vtype, ngf, 0,
                                          t ? hv_partial_blocks(t, vtype) : 1, false, nullptr,
                                          nullptr));
  }
  gdev = reinterpret_cast<double*>(base + off);
  double* cdev = gdev + 2 * kMaxLmats;
  std::vector<double> coeff(4 * (ngf + 1), 0.0);
  for (int br = 0; br < 2; ++br) {
    if (nlen[br] == 0) continue;
    std::copy(ha[br].begin(), ha[br].begin() + nlen[br], coeff.begin() + (2 * br) * (ngf + 1));
    std::copy(hb[br].begin() + 1, hb[br].begin() + 1 + nlen[br],
              coeff.begin() + (2 * br + 1) * (ngf + 1));
  }
  EDX_HIP(hipMemcpyAsync(cdev, coeff.data(), sizeof(double) * coeff.size(), hipMemcpyHostToDevice,
                         st));
  EDX_TRY(k_green_cf(cdev, cdev + (ngf + 1), nlen[0], w[0], cdev + 2 * (ngf + 1),
                     cdev + 3 * (ngf + 1), nlen[1], w[1], e0, o->beta, o->lmats, gdev, st));
  EDX_HIP(hipMemcpyAsync(g_host, gdev, sizeof(double) * 2 * o->lmats, hipMemcpyDeviceToHost, st));
  EDX_HIP(hipStreamSynchronize(st));
  if (rep) {
    rep->wp = w[0];
    rep->wh = w[1];
    rep->np = nlen[0];
    rep->nh = nlen[1];
    for (int br = 0; br < 2; ++br) {
      double* ao = br == 0 ? rep->alpha_p : rep->alpha_h;
      double* bo = br == 0 ? rep->beta_p : rep->beta_h;
      for (int k = 0; k < ngf; ++k) {
        if (ao) ao[k] = k < nlen[br] ? ha[br][k] : 0.0;
        if (bo) bo[k] = k + 1 < nlen[br] ? hb[br][k + 1] : 0.0;
      }
    }
  }
  return EDX_OK;
}

// ---------------------------------------------------------------- susceptibility
size_t chi_workspace_bytes(const edx_sector* s, int vtype, int ngf) {
  return lanczos_ws_layout(s->vlen, vtype, ngf, 0, hv_partial_blocks(s, vtype), false, nullptr,
                           nullptr) + 512;
}

// O psi0 - <O> psi0 for a Hermitian operator that keeps the sector: op 0 the
// diagonal density operator c, op 1 the excitonic operator of levels (a, b)
static edx_status chi_start(const edx_sector* s, int vtype, const void* psi0, int op,
                            const DiagCoef& c, int a, int b, void* phi, double* partial,
                            double* mean, int nb, hipStream_t st) {
  if (op == 0) {
    EDX_TRY(k_diag_apply(s, vtype, psi0, phi, c, nullptr, partial, nb, st));
    EDX_TRY(k_reduce(partial, nb, 1, mean, st));
    return k_diag_apply(s, vtype, psi0, phi, c, mean, partial, nb, st);
  }
  EDX_TRY(k_exc_apply(s, vtype, psi0, phi, a, b, nullptr, partial, nb, st));
  EDX_TRY(k_reduce(partial, nb, 1, mean, st));
  return k_exc_apply(s, vtype, psi0, phi, a, b, mean, partial, nb, st);
}

edx_status chi_impl(const edx_sector* s, const void* psi0, double e0, const DiagCoef& c,
                    const edx_gf_opts* o, void* ws, size_t ws_bytes, double* chi_host,
                    edx_chi_report* rep, hipStream_t st, int op, int a, int b) {
  const int vtype = o->vtype;
  const int ngf = o->ngf;
  if (o->lmats < 1 || o->lmats > kMaxLmats || ngf < 1 || !(o->beta > 0.0)) {
    set_error("chi: need 1 <= lmats <= 65536, ngf >= 1, beta > 0");
    return EDX_E_INVALID;
  }
  LanczosWs L;
  char* base = reinterpret_cast<char*>(align_up(reinterpret_cast<uintptr_t>(ws)));
  const size_t need = lanczos_ws_layout(s->vlen, vtype, ngf, 0, hv_partial_blocks(s, vtype),
                                        false, base, &L);
  if (need + (size_t)(base - (char*)ws) > ws_bytes) {
    set_error("chi: workspace too small (need " + std::to_string(need + 512) + " bytes)");
    return EDX_E_NOMEM;
  }
  const int64_t n = s->vlen;
  const int nb = elem_blocks(n);
  // phi_0 = (O - <O>) psi0 in the padded layout
  EDX_TRY(chi_start(s, vtype, psi0, op, c, a, b, L.vec, L.partial, L.coef, nb, st));
  EDX_TRY(k_beta_finish(L.partial, nb, L.beta, L.scale, st));
  double h[2] = {0.0, 0.0};
  EDX_HIP(hipMemcpyAsync(h, L.beta, sizeof(double), hipMemcpyDeviceToHost, st));
  EDX_HIP(hipMemcpyAsync(h + 1, L.coef, sizeof(double), hipMemcpyDeviceToHost, st));
  EDX_HIP(hipStreamSynchronize(st));
  const double wgt = h[0] * h[0];
  std::fill(chi_host, chi_host + 2 * (size_t)o->lmats, 0.0);
  int len = 0, dropped = 0;
  if (h[0] > 0.0) {
    EDX_HIP(hipMemsetAsync(L.beta, 0, sizeof(double), st));
    for (int j = 0; j < ngf; ++j)
      EDX_TRY(lanczos_step(s, vtype, L, j, 0, L.alpha, L.beta, L.scale, nullptr, nullptr, st));
    std::vector<double> ha(ngf + 1), hb(ngf + 1);
    EDX_HIP(hipMemcpyAsync(ha.data(), L.alpha, sizeof(double) * ngf, hipMemcpyDeviceToHost, st));
    EDX_HIP(hipMemcpyAsync(hb.data(), L.beta, sizeof(double) * (ngf + 1), hipMemcpyDeviceToHost,
                           st));
    EDX_HIP(hipStreamSynchronize(st));
    // truncate at the first breakdown (as for the Green's function)
    double tn = 0.0;
    len = ngf;
    for (int j = 0; j < ngf; ++j) {
      tn = std::max(tn, std::fabs(ha[j]) + hb[j] + hb[j + 1]);
      if (j + 1 < ngf && !(hb[j + 1] > 1e-12 * tn)) {
        len = j + 1;
        break;
      }
    }
    std::vector<double> th(len), wt(len);
    if (!tridiag_spectrum(ha.data(), hb.data() + 1, len, th.data(), wt.data())) {
      set_error("chi: tridiagonal QR did not converge");
      return EDX_E_NOCONV;
    }
    double thr = 1e-9 * std::max(1.0, std::fabs(e0));
    if (vtype == EDX_F32) thr = std::max(thr, 2.0 * 1.1920929e-7 * tn);
    std::vector<double> dd, ww;
    for (int k = 0; k < len; ++k) {
      const double d = th[k] - e0;
      if (std::fabs(d) <= thr) {
        ++dropped;
        continue;
      }
      dd.push_back(d);
      ww.push_back(wgt * wt[k]);
    }
    // 1/(i nu - d) - 1/(i nu + d) = -2 d / (nu^2 + d^2): real
    for (int q = 0; q < o->lmats; ++q) {
      const double nu = 2.0 * q * M_PI / o->beta;
      double acc = 0.0;
      for (size_t k = 0; k < dd.size(); ++k) acc -= 2.0 * ww[k] * dd[k] / (nu * nu + dd[k] * dd[k]);
      chi_host[2 * q] = acc;
    }
  }
  if (rep) {
    rep->w = wgt;
    rep->mean = h[1];
    rep->n = len;
    rep->dropped = dropped;
  }
  return EDX_OK;
}

// ---------------------------------------------------------------- pair susceptibility
// Sectors reached by the pair operators of orbital a: (N_up + 1, N_dw + 1) for
// c+_{a up} c+_{a dw} (k = 0) and (N_up - 1, N_dw - 1) for c_{a dw} c_{a up}
// (k = 1); in an orbital-resolved sector only orbital a's two counts change.
static edx_status ensure_pair_neighbours(const edx_sector* gs, int a, hipStream_t st) {
  edx_sector* g = const_cast<edx_sector*>(gs);
  std::lock_guard<std::mutex> lk(g->nb_mu);
  edx_sector** slot = g->nb_pair[g->orb ? a : 0];
  const Allocator* alloc = gs->alloc.alloc ? &gs->alloc : nullptr;
  for (int k = 0; k < 2; ++k) {
    if (slot[k]) continue;
    const int d = k == 0 ? 1 : -1;
    edx_sector* t = nullptr;
    if (gs->orb) {
      int cu[kMaxNorb], cd[kMaxNorb];
      for (int q = 0; q < kMaxNorb; ++q) {
        cu[q] = gs->up.counts[q];
        cd[q] = gs->dw.counts[q];
      }
      cu[a] += d;
      cd[a] += d;
      const int top = gs->model.nbath + 1;
      if (cu[a] < 0 || cd[a] < 0 || cu[a] > top || cd[a] > top) continue;
      EDX_TRY(build_sector_impl(gs->model, gs->nup + d, gs->ndw + d, st, &t, alloc, cu, cd));
    } else {
      const int nu = gs->nup + d, nd = gs->ndw + d;
      if (nu < 0 || nd < 0 || nu > gs->model.ns || nd > gs->model.ns) continue;
      EDX_TRY(build_sector_impl(gs->model, nu, nd, st, &t, alloc));
    }
    slot[k] = t;
  }
  return EDX_OK;
}

size_t pair_workspace_bytes(const edx_sector* s, int vtype, int ngf) {
  auto comb = [](int nn, int k) -> int64_t {
    if (k < 0 || k > nn) return 0;
    int64_t r = 1;
    for (int i = 1; i <= k; ++i) r = r * (nn - k + i) / i;
    return r;
  };
  const int ns = s->model.ns;
  int64_t dmax = 1, ddw_max = 1;
  for (int d : {-1, 1}) {
    dmax = std::max(dmax, vec_ld(comb(ns, s->nup + d)) * comb(ns, s->ndw + d));
    ddw_max = std::max(ddw_max, comb(ns, s->ndw + d));
  }
  const int hvb = (int)std::max<int64_t>(kMaxPartials, ddw_max + 8 + kNdMaxBlocks);
  return lanczos_ws_layout(dmax, vtype, ngf, 0, hvb, false, nullptr, nullptr) +
         sizeof(double) * (2 * kMaxLmats + 4 * (ngf + 1)) + 512;
}

edx_status pair_impl(const edx_sector* gs, const void* psi0, double e0, int a,
                     const edx_gf_opts* o, void* ws, size_t ws_bytes, double* chi_host,
                     edx_gf_report* rep, hipStream_t st) {
  const int vtype = o->vtype;
  const int ngf = o->ngf;
  if (o->lmats < 1 || o->lmats > kMaxLmats || ngf < 1 || !(o->beta > 0.0)) {
    set_error("chi_pair: need 1 <= lmats <= 65536, ngf >= 1, beta > 0");
    return EDX_E_INVALID;
  }
  const size_t need = pair_workspace_bytes(gs, vtype, ngf);
  if (need > ws_bytes) {
    set_error("chi_pair: workspace too small (need " + std::to_string(need) + " bytes)");
    return EDX_E_NOMEM;
  }
  EDX_TRY(ensure_pair_neighbours(gs, a, st));
  edx_sector* const* nbs = gs->nb_pair[gs->orb ? a : 0];
  char* base = reinterpret_cast<char*>(align_up(reinterpret_cast<uintptr_t>(ws)));
  double w[2] = {0.0, 0.0};
  int nlen[2] = {0, 0};
  std::vector<double> ha[2], hb[2];
  for (int br = 0; br < 2; ++br) {
    const edx_sector* t = nbs[br];
    if (!t) continue;
    LanczosWs L;
    lanczos_ws_layout(t->vlen, vtype, ngf, 0, hv_partial_blocks(t, vtype), false, base, &L);
    EDX_TRY(k_pair_apply(gs, t, vtype, psi0, L.vec, a, br == 0 ? 1 : 0, st));
    EDX_TRY(k_norm2(vtype, L.vec, t->vlen, L.partial, st));
    EDX_TRY(k_beta_finish(L.partial, elem_blocks(t->vlen), L.beta, L.scale, st));
    double nrm = 0.0;
    EDX_HIP(hipMemcpyAsync(&nrm, L.beta, sizeof(double), hipMemcpyDeviceToHost, st));
    EDX_HIP(hipStreamSynchronize(st));
    w[br] = nrm * nrm;
    if (!(nrm > 0.0)) continue;
    EDX_HIP(hipMemsetAsync(L.beta, 0, sizeof(double), st));
    for (int j = 0; j < ngf; ++j)
      EDX_TRY(lanczos_step(t, vtype, L, j, 0, L.alpha, L.beta, L.scale, nullptr, nullptr, st));
    ha[br].resize(ngf + 1);
    hb[br].resize(ngf + 1);
    EDX_HIP(hipMemcpyAsync(ha[br].data(), L.alpha, sizeof(double) * ngf, hipMemcpyDeviceToHost, st));
    EDX_HIP(hipMemcpyAsync(hb[br].data(), L.beta, sizeof(double) * (ngf + 1), hipMemcpyDeviceToHost,
                           st));
    EDX_HIP(hipStreamSynchronize(st));
    double tn = 0.0;
    int len = ngf;
    for (int j = 0; j < ngf; ++j) {
      tn = std::max(tn, std::fabs(ha[br][j]) + hb[br][j] + hb[br][j + 1]);
      if (j + 1 < ngf && !(hb[br][j + 1] > 1e-12 * tn)) {
        len = j + 1;
        break;
      }
    }
    nlen[br] = len;
  }
  size_t off = 0;
  for (int br = 0; br < 2; ++br) {
    const edx_sector* t = nbs[br];
    off = std::max(off, lanczos_ws_layout(t ? t->vlen : 1, vtype, ngf, 0,
                                          t ? hv_partial_blocks(t, vtype) : 1, false, nullptr,
                                          nullptr));
  }
  double* gdev = reinterpret_cast<double*>(base + off);
  double* cdev = gdev + 2 * kMaxLmats;
  std::vector<double> coeff(4 * (ngf + 1), 0.0);
  for (int br = 0; br < 2; ++br) {
    if (nlen[br] == 0) continue;
    std::copy(ha[br].begin(), ha[br].begin() + nlen[br], coeff.begin() + (2 * br) * (ngf + 1));
    std::copy(hb[br].begin() + 1, hb[br].begin() + 1 + nlen[br],
              coeff.begin() + (2 * br + 1) * (ngf + 1));
  }
  EDX_HIP(hipMemcpyAsync(cdev, coeff.data(), sizeof(double) * coeff.size(), hipMemcpyHostToDevice,
                         st));
  // bosonic: the hole branch enters with a minus sign, nu_n = 2 n pi / beta
  EDX_TRY(k_green_cf(cdev, cdev + (ngf + 1), nlen[0], w[0], cdev + 2 * (ngf + 1),
                     cdev + 3 * (ngf + 1), nlen[1], -w[1], e0, o->beta, o->lmats, gdev, st, 1));
  EDX_HIP(hipMemcpyAsync(chi_host, gdev, sizeof(double) * 2 * o->lmats, hipMemcpyDeviceToHost, st));
  EDX_HIP(hipStreamSynchronize(st));
  if (rep) {
    rep->wp = w[0];
    rep->wh = w[1];
    rep->np = nlen[0];
    rep->nh = nlen[1];
  }
  return EDX_OK;
}

}  // namespace edx
