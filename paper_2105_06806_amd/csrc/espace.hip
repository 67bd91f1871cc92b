// Eigenstate list for finite temperature (Sec. 6 "Eigenspace class") and the
// thermal Green's function (Sec. 6 "Dynamical correlation functions", the
// Boltzmann-weighted sum over states).
//
// Host-side bookkeeping around two device paths that already exist: the k
// lowest states of a sector (lowest_states_impl: Lanczos with full
// re-orthogonalisation and locking) and the Krylov continued fraction of one
// state (green_cf_impl).  The paper keeps the states in an ordered linked
// list; here a sorted array of (energy, sector slot, state index) is rebuilt at
// every diagonalisation, and the vectors stay where the sector's solve wrote
// them: one device block per sector, states one after another, so the kept
// states of a sector are always its lowest ones and need no copy.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <string>
#include <thread>
#include <vector>

#include "edx_internal.h"

struct edx_espace {
  edx_espace_opts o{};
  int nsec = 0;
  int vtype = EDX_F64;
  std::vector<const edx_sector*> secs;   // slots of the last diagonalisation
  std::vector<int> next, computed, kept;
  std::vector<void*> buf;                // per slot: computed vectors, dense
  struct State {
    double e;
    int sec;
    int idx;
  };
  std::vector<State> list;               // kept states, ascending energy
  double e0 = 0.0, z = 0.0;
};

namespace edx {
namespace {

// sectors solved concurrently by edx_espace_diag (one stream and host thread
// each): small sectors are bound by launch and synchronisation latency, which
// the other streams' work hides
constexpr int kEspaceStreams = 3;

edx_status invalid_e(const std::string& msg) {
  set_error(msg);
  return EDX_E_INVALID;
}

// Runs fn(n, stream, workspace part, t) for every kept state n on up to
// kEspaceStreams host threads and streams, state n on thread n % T (a fixed
// assignment, so per-thread sums are reproducible).  ws holds T parts of
// `part` bytes; the caller's stream is thread 0's.
template <class F>
edx_status for_kept_states(const edx_espace* E, void* ws, size_t ws_bytes, size_t part,
                           hipStream_t st, int* nthr_out, F fn) {
  const int ns = (int)E->list.size();
  const int T = (int)std::min<size_t>({(size_t)kEspaceStreams, (size_t)ns,
                                       part ? ws_bytes / part : 1});
  if (T < 1) {
    set_error("espace: workspace too small (need " + std::to_string(part) + " bytes)");
    return EDX_E_NOMEM;
  }
  *nthr_out = T;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipStreamSynchronize(st) != hipSuccess) {
    set_error("espace: device query failed");
    return EDX_E_DEVICE;
  }
  std::vector<hipStream_t> sts(T, st);
  for (int t = 1; t < T; ++t)
    if (hipStreamCreateWithFlags(&sts[t], hipStreamNonBlocking) != hipSuccess) {
      for (int q = 1; q < t; ++q) (void)hipStreamDestroy(sts[q]);
      set_error("espace: stream set-up failed");
      return EDX_E_DEVICE;
    }
  std::vector<edx_status> tst(T, EDX_OK);
  std::vector<std::string> terr(T);
  std::atomic<bool> stop{false};
  auto worker = [&](int t) {
    if (t > 0 && hipSetDevice(dev) != hipSuccess) {
      tst[t] = EDX_E_DEVICE;
      terr[t] = "espace: hipSetDevice failed in a helper thread";
      stop.store(true);
      return;
    }
    char* wsp = static_cast<char*>(ws) + (size_t)t * part;
    for (int n = t; n < ns && !stop.load(); n += T) {
      const edx_status rc = fn(n, sts[t], wsp, t);
      if (rc != EDX_OK) {
        tst[t] = rc;
        terr[t] = edx_last_error();
        stop.store(true);
        break;
      }
    }
  };
  std::vector<std::thread> th;
  for (int t = 1; t < T; ++t) th.emplace_back(worker, t);
  worker(0);
  for (auto& x : th) x.join();
  for (int t = 1; t < T; ++t) {
    (void)hipStreamSynchronize(sts[t]);
    (void)hipStreamDestroy(sts[t]);
  }
  for (int t = 0; t < T; ++t)
    if (tst[t] != EDX_OK) {
      set_error(terr[t]);
      return tst[t];
    }
  return EDX_OK;
}

void release(edx_espace* E) {
  for (auto& p : E->buf)
    if (p) {
      (void)hipFree(p);
      p = nullptr;
    }
  E->list.clear();
  E->e0 = 0.0;
  E->z = 0.0;
}

}  // namespace
}  // namespace edx

using namespace edx;

extern "C" {

void edx_espace_default_opts(edx_espace_opts* o) {
  if (!o) return;
  o->beta = 1000.0;
  o->cutoff = 1e-9;
  o->nstates_sector = 2;
  o->nstates_total = 1;
  o->nstates_step = 2;
  o->verify = 1;
}

edx_status edx_espace_create(const edx_espace_opts* o, int32_t nsec, edx_espace** out) {
  if (!out) return invalid_e("out is NULL");
  *out = nullptr;
  if (!o) return invalid_e("opts is NULL");
  if (!(o->beta > 0.0) || !std::isfinite(o->beta)) return invalid_e("beta must be finite and > 0");
  if (!(o->cutoff >= 0.0 && o->cutoff <= 1.0)) return invalid_e("cutoff must be in [0, 1]");
  if (o->nstates_sector < 1 || o->nstates_sector > EDX_MAX_STATES)
    return invalid_e("nstates_sector must be in [1, 64]");
  if (o->nstates_total < 1) return invalid_e("nstates_total must be >= 1");
  if (o->nstates_step < 0) return invalid_e("nstates_step must be >= 0");
  if (nsec < 1) return invalid_e("nsec must be >= 1");
  edx_espace* E = new edx_espace();
  E->o = *o;
  E->nsec = nsec;
  E->next.assign(nsec, o->nstates_sector);
  E->computed.assign(nsec, 0);
  E->kept.assign(nsec, 0);
  E->buf.assign(nsec, nullptr);
  E->secs.assign(nsec, nullptr);
  *out = E;
  return EDX_OK;
}

void edx_espace_destroy(edx_espace* E) {
  if (!E) return;
  release(E);
  delete E;
}

size_t edx_espace_diag_workspace_bytes(const edx_espace* E, edx_sector* const* secs, int32_t nsec,
                                       int32_t vtype, int32_t niter) {
  if (!E || !secs || nsec != E->nsec || (vtype != EDX_F64 && vtype != EDX_F32) || niter < 1)
    return 0;
  size_t need = 0;
  for (int i = 0; i < nsec; ++i) {
    if (!secs[i]) return 0;
    need = std::max(need, lowest_workspace_bytes(secs[i], vtype, niter, E->next[i]));
  }
  return align_up(need) * (size_t)std::min(kEspaceStreams, (int)nsec);
}

edx_status edx_espace_diag(edx_espace* E, edx_sector* const* secs, int32_t nsec,
                           const edx_lanczos_opts* o, void* ws, size_t ws_bytes, void* stream) {
  if (!E || !secs || !o || !ws) return invalid_e("espace, secs, opts and ws must be non-NULL");
  if (nsec != E->nsec) return invalid_e("nsec differs from the espace's sector count");
  for (int i = 0; i < nsec; ++i)
    if (!secs[i]) return invalid_e("a sector handle is NULL");
  if (o->vtype != EDX_F64 && o->vtype != EDX_F32) return invalid_e("vtype must be EDX_F64 or EDX_F32");
  if (o->niter < 1 || o->niter > 4096) return invalid_e("niter must be in [1, 4096]");
  if (!(o->tol >= 0.0) || !(o->rtol >= 0.0) || !(o->tol > 0.0 || o->rtol > 0.0))
    return invalid_e("tol/rtol must be >= 0, one of them > 0");
  hipStream_t st = static_cast<hipStream_t>(stream);
  release(E);
  E->vtype = o->vtype;
  E->secs.assign(secs, secs + nsec);
  // one workspace part per stream
  size_t part = 0;
  for (int i = 0; i < nsec; ++i)
    part = std::max(part, align_up(lowest_workspace_bytes(secs[i], o->vtype, o->niter,
                                                          E->next[i])));
  const int nthr = (int)std::min<size_t>({(size_t)kEspaceStreams, (size_t)nsec,
                                          part ? ws_bytes / part : 1});
  if (nthr < 1) {
    set_error("espace: workspace too small (need " + std::to_string(part) + " bytes)");
    return EDX_E_NOMEM;
  }
  std::vector<int> kreq(nsec);
  for (int i = 0; i < nsec; ++i) {
    const edx_sector* s = secs[i];
    kreq[i] = (int)std::min<int64_t>(E->next[i], s->dim);
    void* p = nullptr;
    if (hipMalloc(&p, (size_t)kreq[i] * s->dim * vbytes(o->vtype)) != hipSuccess) {
      (void)hipGetLastError();
      release(E);
      set_error("espace: out of device memory for the state vectors");
      return EDX_E_NOMEM;
    }
    E->buf[i] = p;
  }
  // largest sectors first, pulled by the workers from a shared counter
  std::vector<int> order(nsec);
  for (int i = 0; i < nsec; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(),
                   [&](int x, int y) { return secs[x]->dim > secs[y]->dim; });
  std::vector<std::vector<double>> ev(nsec);
  std::vector<int> found(nsec, 0);
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipStreamSynchronize(st) != hipSuccess) {
    release(E);
    set_error("espace: device query failed");
    return EDX_E_DEVICE;
  }
  std::vector<hipStream_t> sts(nthr, st);
  edx_status fail = EDX_OK;
  for (int t = 1; t < nthr; ++t)
    if (hipStreamCreateWithFlags(&sts[t], hipStreamNonBlocking) != hipSuccess) {
      sts[t] = st;
      fail = EDX_E_DEVICE;
    }
  std::atomic<int> next{0};
  std::vector<edx_status> tst(nthr, EDX_OK);
  std::vector<std::string> terr(nthr);
  auto worker = [&](int t) {
    if (t > 0 && hipSetDevice(dev) != hipSuccess) {
      tst[t] = EDX_E_DEVICE;
      terr[t] = "espace: hipSetDevice failed in a helper thread";
      next.store(nsec);
      return;
    }
    char* wsp = static_cast<char*>(ws) + (size_t)t * part;
    for (;;) {
      const int q = next.fetch_add(1);
      if (q >= nsec) break;
      const int i = order[q];
      ev[i].assign(kreq[i], 0.0);
      edx_lowest_report r{};
      const edx_status rc = lowest_states_impl(secs[i], kreq[i], o, E->o.verify, wsp, part,
                                               ev[i].data(), E->buf[i], &r, sts[t]);
      if (rc != EDX_OK) {
        tst[t] = rc;
        terr[t] = edx_last_error();
        next.store(nsec);
        break;
      }
      found[i] = r.nfound;
    }
  };
  if (fail == EDX_OK) {
    std::vector<std::thread> th;
    for (int t = 1; t < nthr; ++t) th.emplace_back(worker, t);
    worker(0);
    for (auto& x : th) x.join();
  }
  for (int t = 1; t < nthr; ++t)
    if (sts[t] != st) {
      (void)hipStreamSynchronize(sts[t]);
      (void)hipStreamDestroy(sts[t]);
    }
  for (int t = 0; t < nthr && fail == EDX_OK; ++t)
    if (tst[t] != EDX_OK) {
      fail = tst[t];
      set_error(terr[t]);
    }
  if (fail != EDX_OK) {
    release(E);
    if (fail == EDX_E_DEVICE && edx_last_error()[0] == 0) set_error("espace: stream set-up failed");
    return fail;
  }
  std::vector<edx_espace::State> all;
  for (int i = 0; i < nsec; ++i) {
    E->computed[i] = found[i];
    for (int j = 0; j < found[i]; ++j) all.push_back({ev[i][j], i, j});
  }
  std::stable_sort(all.begin(), all.end(), [](const edx_espace::State& a, const edx_espace::State& b) {
    if (a.e != b.e) return a.e < b.e;
    if (a.sec != b.sec) return a.sec < b.sec;
    return a.idx < b.idx;
  });
  std::fill(E->kept.begin(), E->kept.end(), 0);
  if (!all.empty()) {
    E->e0 = all[0].e;
    for (const auto& t : all) {
      if ((int)E->list.size() >= E->o.nstates_total) break;
      const double f = std::exp(-E->o.beta * (t.e - E->e0));
      if (!(f >= E->o.cutoff)) break;   // ascending energies: every later factor is smaller
      E->list.push_back(t);
      E->kept[t.sec] += 1;
      E->z += f;
    }
  }
  for (int i = 0; i < nsec; ++i) {
    const int c = E->computed[i], kk = E->kept[i];
    const int nx = (c > 0 && kk == c) ? E->next[i] + E->o.nstates_step : std::max(1, kk);
    E->next[i] = std::min(nx, EDX_MAX_STATES);
    if (kk == 0 && E->buf[i]) {
      (void)hipFree(E->buf[i]);
      E->buf[i] = nullptr;
    }
  }
  return EDX_OK;
}

edx_status edx_espace_info(const edx_espace* E, int32_t* nstates, double* e0, double* z) {
  if (!E) return invalid_e("espace is NULL");
  if (nstates) *nstates = (int32_t)E->list.size();
  if (e0) *e0 = E->e0;
  if (z) *z = E->z;
  return EDX_OK;
}

edx_status edx_espace_state(const edx_espace* E, int32_t i, double* e, int32_t* sec,
                            double* weight, const void** psi) {
  if (!E) return invalid_e("espace is NULL");
  if (i < 0 || i >= (int)E->list.size()) return invalid_e("state index out of range");
  const auto& t = E->list[i];
  if (e) *e = t.e;
  if (sec) *sec = t.sec;
  if (weight) *weight = std::exp(-E->o.beta * (t.e - E->e0)) / E->z;
  if (psi)
    *psi = static_cast<const char*>(E->buf[t.sec]) +
           (size_t)t.idx * E->secs[t.sec]->dim * vbytes(E->vtype);
  return EDX_OK;
}

edx_status edx_espace_sector(const edx_espace* E, int32_t sec, int32_t* computed, int32_t* kept,
                             int32_t* next) {
  if (!E) return invalid_e("espace is NULL");
  if (sec < 0 || sec >= E->nsec) return invalid_e("sector slot out of range");
  if (computed) *computed = E->computed[sec];
  if (kept) *kept = E->kept[sec];
  if (next) *next = E->next[sec];
  return EDX_OK;
}

size_t edx_espace_green_workspace_bytes(const edx_espace* E, int32_t ngf) {
  if (!E || ngf < 1) return 0;
  size_t need = 0;
  for (int i = 0; i < E->nsec; ++i)
    if (E->kept[i] > 0 && E->secs[i])
      need = std::max(need, green_workspace_bytes(E->secs[i], E->vtype, ngf));
  return align_up(need) * (size_t)std::max(1, std::min(kEspaceStreams, (int)E->list.size()));
}

edx_status edx_espace_green(edx_espace* E, int32_t orb, int32_t spin, const edx_gf_opts* o,
                            void* ws, size_t ws_bytes, double* g_host, void* stream) {
  if (!E || !o || !ws || !g_host) return invalid_e("espace, opts, ws and g_host must be non-NULL");
  if (E->list.empty()) return invalid_e("the state list is empty (run edx_espace_diag first)");
  if (o->vtype != E->vtype) return invalid_e("opts->vtype differs from the stored vectors' type");
  if (std::fabs(o->beta - E->o.beta) > 1e-12 * E->o.beta)
    return invalid_e("opts->beta differs from the espace's beta");
  if (spin != 0 && spin != 1) return invalid_e("spin must be 0 or 1");
  if (o->ngf < 1 || o->ngf > 4096) return invalid_e("ngf must be in [1, 4096]");
  const int lm = o->lmats;
  if (lm < 1) return invalid_e("lmats must be >= 1");
  for (const auto& t : E->list)
    if (orb < 0 || orb >= E->secs[t.sec]->model.norb) return invalid_e("orb out of range");
  size_t part = 0;
  for (int i = 0; i < E->nsec; ++i)
    if (E->kept[i] > 0) part = std::max(part, align_up(green_workspace_bytes(E->secs[i], E->vtype, o->ngf)));
  // per-thread sums (state n on thread n % T), added in thread order
  std::vector<std::vector<double>> acc(kEspaceStreams, std::vector<double>(2 * (size_t)lm, 0.0));
  std::vector<std::vector<double>> gn(kEspaceStreams, std::vector<double>(2 * (size_t)lm));
  int T = 1;
  EDX_TRY(for_kept_states(E, ws, ws_bytes, part, static_cast<hipStream_t>(stream), &T,
                          [&](int n, hipStream_t st, void* wsp, int th) -> edx_status {
    const auto& t = E->list[n];
    const edx_sector* s = E->secs[t.sec];
    const void* psi =
        static_cast<const char*>(E->buf[t.sec]) + (size_t)t.idx * s->dim * vbytes(E->vtype);
    EDX_TRY(green_cf_impl(s, psi, t.e, orb, spin, o, wsp, part, gn[th].data(), nullptr, st));
    const double w = std::exp(-E->o.beta * (t.e - E->e0)) / E->z;
    for (size_t q = 0; q < acc[th].size(); ++q) acc[th][q] += w * gn[th][q];
    return EDX_OK;
  }));
  for (size_t q = 0; q < 2 * (size_t)lm; ++q) {
    double x = 0.0;
    for (int th = 0; th < T; ++th) x += acc[th][q];
    g_host[q] = x;
  }
  return EDX_OK;
}

size_t edx_espace_chi_workspace_bytes(const edx_espace* E, int32_t ngf) {
  if (!E || ngf < 1) return 0;
  size_t need = 0;
  for (int i = 0; i < E->nsec; ++i)
    if (E->kept[i] > 0 && E->secs[i])
      need = std::max(need, chi_workspace_bytes(E->secs[i], E->vtype, ngf));
  return align_up(need) * (size_t)std::max(1, std::min(kEspaceStreams, (int)E->list.size()));
}

edx_status edx_espace_chi(edx_espace* E, const double* cu, const double* cd,
                          const edx_gf_opts* o, void* ws, size_t ws_bytes, double* chi_host,
                          void* stream) {
  if (!E || !cu || !cd || !o || !ws || !chi_host)
    return invalid_e("espace, cu, cd, opts, ws and chi_host must be non-NULL");
  if (E->list.empty()) return invalid_e("the state list is empty (run edx_espace_diag first)");
  if (o->vtype != E->vtype) return invalid_e("opts->vtype differs from the stored vectors' type");
  if (std::fabs(o->beta - E->o.beta) > 1e-12 * E->o.beta)
    return invalid_e("opts->beta differs from the espace's beta");
  if (o->ngf < 1 || o->ngf > 4096) return invalid_e("ngf must be in [1, 4096]");
  const int lm = o->lmats;
  if (lm < 1) return invalid_e("lmats must be >= 1");
  size_t part = 0;
  for (int i = 0; i < E->nsec; ++i)
    if (E->kept[i] > 0) part = std::max(part, align_up(chi_workspace_bytes(E->secs[i], E->vtype, o->ngf)));
  std::vector<std::vector<double>> acc(kEspaceStreams, std::vector<double>(2 * (size_t)lm, 0.0));
  std::vector<std::vector<double>> cn(kEspaceStreams, std::vector<double>(2 * (size_t)lm));
  int T = 1;
  EDX_TRY(for_kept_states(E, ws, ws_bytes, part, static_cast<hipStream_t>(stream), &T,
                          [&](int n, hipStream_t st, void* wsp, int th) -> edx_status {
    const auto& t = E->list[n];
    const edx_sector* s = E->secs[t.sec];
    DiagCoef c{};
    for (int a = 0; a < s->model.norb; ++a) {
      c.up[a] = cu[a];
      c.dw[a] = cd[a];
    }
    const void* psi =
        static_cast<const char*>(E->buf[t.sec]) + (size_t)t.idx * s->dim * vbytes(E->vtype);
    EDX_TRY(chi_impl(s, psi, t.e, c, o, wsp, part, cn[th].data(), nullptr, st));
    const double w = std::exp(-E->o.beta * (t.e - E->e0)) / E->z;
    for (size_t q = 0; q < acc[th].size(); ++q) acc[th][q] += w * cn[th][q];
    return EDX_OK;
  }));
  for (size_t q = 0; q < 2 * (size_t)lm; ++q) {
    double x = 0.0;
    for (int th = 0; th < T; ++th) x += acc[th][q];
    chi_host[q] = x;
  }
  return EDX_OK;
}

size_t edx_espace_pair_workspace_bytes(const edx_espace* E, int32_t ngf) {
  if (!E || ngf < 1) return 0;
  size_t need = 0;
  for (int i = 0; i < E->nsec; ++i)
    if (E->kept[i] > 0 && E->secs[i])
      need = std::max(need, pair_workspace_bytes(E->secs[i], E->vtype, ngf));
  return align_up(need) * (size_t)std::max(1, std::min(kEspaceStreams, (int)E->list.size()));
}

// thermal sum of a per-state function: kind 0 exciton (a, b), 1 pair (a)
static edx_status espace_op_sum(edx_espace* E, int kind, int a, int b, const edx_gf_opts* o,
                                void* ws, size_t ws_bytes, double* out, void* stream) {
  if (!E || !o || !ws || !out) return invalid_e("espace, opts, ws and output must be non-NULL");
  if (E->list.empty()) return invalid_e("the state list is empty (run edx_espace_diag first)");
  if (o->vtype != E->vtype) return invalid_e("opts->vtype differs from the stored vectors' type");
  if (std::fabs(o->beta - E->o.beta) > 1e-12 * E->o.beta)
    return invalid_e("opts->beta differs from the espace's beta");
  if (o->ngf < 1 || o->ngf > 4096) return invalid_e("ngf must be in [1, 4096]");
  const int lm = o->lmats;
  if (lm < 1) return invalid_e("lmats must be >= 1");
  size_t part = 0;
  for (const auto& t : E->list) {
    const edx_sector* s = E->secs[t.sec];
    const int norb = s->model.norb;
    if (kind == 0 && (a < 0 || b < 0 || a >= norb || b >= norb || a == b))
      return invalid_e("a and b must be two different orbitals");
    if (kind == 1 && (a < 0 || a >= norb)) return invalid_e("orbital out of range");
    if (s->dph > 1 || (kind == 0 && s->orb)) {
      set_error("espace: this susceptibility needs sectors without phonons (and total-N for the "
                "excitonic one)");
      return EDX_E_UNSUPPORTED;
    }
    part = std::max(part, align_up(kind == 0 ? chi_workspace_bytes(s, E->vtype, o->ngf)
                                             : pair_workspace_bytes(s, E->vtype, o->ngf)));
  }
  std::vector<std::vector<double>> acc(kEspaceStreams, std::vector<double>(2 * (size_t)lm, 0.0));
  std::vector<std::vector<double>> cn(kEspaceStreams, std::vector<double>(2 * (size_t)lm));
  int T = 1;
  EDX_TRY(for_kept_states(E, ws, ws_bytes, part, static_cast<hipStream_t>(stream), &T,
                          [&](int n, hipStream_t st, void* wsp, int th) -> edx_status {
    const auto& t = E->list[n];
    const edx_sector* s = E->secs[t.sec];
    const void* psi =
        static_cast<const char*>(E->buf[t.sec]) + (size_t)t.idx * s->dim * vbytes(E->vtype);
    if (kind == 0) {
      DiagCoef c{};
      EDX_TRY(chi_impl(s, psi, t.e, c, o, wsp, part, cn[th].data(), nullptr, st, 1,
                       std::min(a, b), std::max(a, b)));
    } else {
      EDX_TRY(pair_impl(s, psi, t.e, a, o, wsp, part, cn[th].data(), nullptr, st));
    }
    const double w = std::exp(-E->o.beta * (t.e - E->e0)) / E->z;
    for (size_t q = 0; q < acc[th].size(); ++q) acc[th][q] += w * cn[th][q];
    return EDX_OK;
  }));
  for (size_t q = 0; q < 2 * (size_t)lm; ++q) {
    double x = 0.0;
    for (int th = 0; th < T; ++th) x += acc[th][q];
    out[q] = x;
  }
  return EDX_OK;
}

edx_status edx_espace_chi_exciton(edx_espace* E, int32_t a, int32_t b, const edx_gf_opts* o,
                                  void* ws, size_t ws_bytes, double* chi_host, void* stream) {
  return espace_op_sum(E, 0, a, b, o, ws, ws_bytes, chi_host, stream);
}

edx_status edx_espace_chi_pair(edx_espace* E, int32_t a, const edx_gf_opts* o, void* ws,
                               size_t ws_bytes, double* chi_host, void* stream) {
  return espace_op_sum(E, 1, a, 0, o, ws, ws_bytes, chi_host, stream);
}

}  // extern "C"
