// Eigenstate list for finite temperature (Sec. 5 "Eigenspace class") and the
// thermal Green's function (Sec. 5 "Dynamical correlation functions", the
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
#include <cmath>
#include <string>
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

edx_status invalid_e(const std::string& msg) {
  set_error(msg);
  return EDX_E_INVALID;
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
  return need;
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
  std::vector<edx_espace::State> all;
  for (int i = 0; i < nsec; ++i) {
    const edx_sector* s = secs[i];
    const int k = (int)std::min<int64_t>(E->next[i], s->dim);
    void* p = nullptr;
    if (hipMalloc(&p, (size_t)k * s->dim * vbytes(o->vtype)) != hipSuccess) {
      (void)hipGetLastError();
      release(E);
      set_error("espace: out of device memory for the state vectors");
      return EDX_E_NOMEM;
    }
    E->buf[i] = p;
    std::vector<double> e(k);
    edx_lowest_report r{};
    const edx_status rc = lowest_states_impl(s, k, o, E->o.verify, ws, ws_bytes, e.data(), p, &r, st);
    if (rc != EDX_OK) {
      release(E);
      return rc;
    }
    E->computed[i] = r.nfound;
    for (int j = 0; j < r.nfound; ++j) all.push_back({e[j], i, j});
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
  return need;
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
  std::vector<double> acc(2 * (size_t)lm, 0.0), gn(2 * (size_t)lm);
  for (int n = 0; n < (int)E->list.size(); ++n) {
    const auto& t = E->list[n];
    const edx_sector* s = E->secs[t.sec];
    if (orb < 0 || orb >= s->model.norb) return invalid_e("orb out of range");
    const void* psi =
        static_cast<const char*>(E->buf[t.sec]) + (size_t)t.idx * s->dim * vbytes(E->vtype);
    EDX_TRY(green_cf_impl(s, psi, t.e, orb, spin, o, ws, ws_bytes, gn.data(), nullptr,
                          static_cast<hipStream_t>(stream)));
    const double w = std::exp(-E->o.beta * (t.e - E->e0)) / E->z;
    for (size_t q = 0; q < acc.size(); ++q) acc[q] += w * gn[q];
  }
  std::copy(acc.begin(), acc.end(), g_host);
  return EDX_OK;
}

size_t edx_espace_chi_workspace_bytes(const edx_espace* E, int32_t ngf) {
  if (!E || ngf < 1) return 0;
  size_t need = 0;
  for (int i = 0; i < E->nsec; ++i)
    if (E->kept[i] > 0 && E->secs[i])
      need = std::max(need, chi_workspace_bytes(E->secs[i], E->vtype, ngf));
  return need;
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
  std::vector<double> acc(2 * (size_t)lm, 0.0), cn(2 * (size_t)lm);
  for (int n = 0; n < (int)E->list.size(); ++n) {
    const auto& t = E->list[n];
    const edx_sector* s = E->secs[t.sec];
    DiagCoef c{};
    for (int a = 0; a < s->model.norb; ++a) {
      c.up[a] = cu[a];
      c.dw[a] = cd[a];
    }
    const void* psi =
        static_cast<const char*>(E->buf[t.sec]) + (size_t)t.idx * s->dim * vbytes(E->vtype);
    EDX_TRY(chi_impl(s, psi, t.e, c, o, ws, ws_bytes, cn.data(), nullptr,
                     static_cast<hipStream_t>(stream)));
    const double w = std::exp(-E->o.beta * (t.e - E->e0)) / E->z;
    for (size_t q = 0; q < acc.size(); ++q) acc[q] += w * cn[q];
  }
  std::copy(acc.begin(), acc.end(), chi_host);
  return EDX_OK;
}

}  // extern "C"
