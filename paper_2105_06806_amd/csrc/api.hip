// extern "C" entry points of libedx (declared in include/edx.h): argument
// checking, error strings and dispatch to the drivers.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>

#include "edx_internal.h"

namespace edx {

namespace {
thread_local std::string g_last_error;
}

void set_error(const std::string& msg) { g_last_error = msg; }

static edx_status invalid(const std::string& msg) {
  set_error(msg);
  return EDX_E_INVALID;
}

static edx_status check_model(const edx_model* m, Model* out) {
  if (!m) return invalid("model is NULL");
  if (m->norb < 1 || m->norb > kMaxNorb) return invalid("norb must be in [1, 3]");
  if (m->nbath < 0) return invalid("nbath must be >= 0");
  const int ns = m->norb * (m->nbath + 1);
  if (ns > kMaxNs) {
    set_error("Ns = norb*(nbath+1) must be <= 24");
    return EDX_E_UNSUPPORTED;
  }
  if (m->norb * m->nbath > 127) {
    set_error("at most 127 hybridisation pairs");
    return EDX_E_UNSUPPORTED;
  }
  if (!m->eps_imp) return invalid("eps_imp is NULL");
  if (m->nbath > 0 && (!m->eps_bath || !m->vhyb)) return invalid("eps_bath/vhyb is NULL");
  out->norb = m->norb;
  out->nbath = m->nbath;
  out->ns = ns;
  out->eps_imp.assign(m->eps_imp, m->eps_imp + m->norb);
  const int nb = m->norb * m->nbath;
  out->eps_bath.assign(m->eps_bath, m->eps_bath + nb);
  out->vhyb.assign(m->vhyb, m->vhyb + nb);
  out->U = m->U;
  out->Ust = m->Ust;
  out->Jh = m->Jh;
  out->xmu = m->xmu;
  out->Jx = m->Jx;
  out->Jp = m->Jp;
  for (double x : out->eps_imp)
    if (!std::isfinite(x)) return invalid("non-finite eps_imp");
  for (double x : out->eps_bath)
    if (!std::isfinite(x)) return invalid("non-finite eps_bath");
  for (double x : out->vhyb)
    if (!std::isfinite(x)) return invalid("non-finite vhyb");
  if (!std::isfinite(m->U) || !std::isfinite(m->Ust) || !std::isfinite(m->Jh) ||
      !std::isfinite(m->xmu) || !std::isfinite(m->Jx) || !std::isfinite(m->Jp))
    return invalid("non-finite interaction parameter");
  if (m->nph < 0 || m->nph > kMaxPh) return invalid("nph must be in [0, 63]");
  out->nph = m->nph;
  if (m->nph > 0) {
    if (!m->g) return invalid("g is NULL with nph > 0");
    if (!std::isfinite(m->w0)) return invalid("non-finite w0");
    out->w0 = m->w0;
    for (int a = 0; a < m->norb; ++a) {
      if (!std::isfinite(m->g[a])) return invalid("non-finite g");
      out->g[a] = m->g[a];
    }
  }
  return EDX_OK;
}

static edx_status check_sector(const edx_sector* s) {
  if (!s) return invalid("sector is NULL");
  int dev = -1;
  EDX_HIP(hipGetDevice(&dev));
  if (dev != s->device) return invalid("sector was built on another device than the current one");
  return EDX_OK;
}

static bool valid_vtype(int v) { return v == EDX_F64 || v == EDX_F32; }

}  // namespace edx

using namespace edx;

extern "C" {

edx_status edx_build_sector(const edx_model* model, int32_t nup, int32_t ndw, void* stream,
                            edx_sector** out) {
  if (!out) return invalid("out is NULL");
  *out = nullptr;
  Model m;
  EDX_TRY(check_model(model, &m));
  if (nup < 0 || ndw < 0 || nup > m.ns || ndw > m.ns)
    return invalid("nup/ndw must be in [0, Ns]");
  return build_sector_impl(m, nup, ndw, static_cast<hipStream_t>(stream), out);
}

edx_status edx_build_sector_orbital(const edx_model* model, const int32_t* nup,
                                    const int32_t* ndw, void* stream, edx_sector** out) {
  if (!out) return invalid("out is NULL");
  *out = nullptr;
  if (!nup || !ndw) return invalid("nup/ndw arrays are NULL");
  Model m;
  EDX_TRY(check_model(model, &m));
  if (m.Jx != 0.0 || m.Jp != 0.0) {
    set_error("orbital-resolved sectors need Jx = Jp = 0 (H_nd mixes orbital counts)");
    return EDX_E_UNSUPPORTED;
  }
  int cu[kMaxNorb] = {0, 0, 0}, cd[kMaxNorb] = {0, 0, 0};
  int su = 0, sd = 0;
  for (int a = 0; a < m.norb; ++a) {
    if (nup[a] < 0 || ndw[a] < 0 || nup[a] > m.nbath + 1 || ndw[a] > m.nbath + 1)
      return invalid("per-orbital counts must be in [0, nbath + 1]");
    cu[a] = nup[a];
    cd[a] = ndw[a];
    su += cu[a];
    sd += cd[a];
  }
  return build_sector_impl(m, su, sd, static_cast<hipStream_t>(stream), out, nullptr, cu, cd);
}

void edx_sector_destroy(edx_sector* s) { destroy_sector(s); }

edx_status edx_sector_dims(const edx_sector* s, int64_t* dup, int64_t* ddw, int64_t* dim) {
  if (!s) return invalid("sector is NULL");
  if (dup) *dup = s->dup;
  if (ddw) *ddw = s->ddw;
  if (dim) *dim = s->dim;
  return EDX_OK;
}

edx_status edx_sector_ld(const edx_sector* s, int64_t* ld) {
  if (!s || !ld) return invalid("sector or ld is NULL");
  *ld = s->ld;
  return EDX_OK;
}

edx_status edx_sector_hop_nnz(const edx_sector* s, int32_t spin, int64_t* nnz, int32_t* max_row) {
  if (!s) return invalid("sector is NULL");
  if (spin != 0 && spin != 1) return invalid("spin must be 0 or 1");
  const SpinTables& T = spin == 0 ? s->up : s->dw;
  if (nnz) *nnz = T.nnz;
  if (max_row) *max_row = T.width;
  return EDX_OK;
}

edx_status edx_sector_get_tables(const edx_sector* s, int32_t spin, uint32_t* map,
                                 int64_t* hop_off, int32_t* hop_col, int8_t* hop_sign,
                                 double* hop_amp, double* diag_e, uint8_t* diag_p) {
  EDX_TRY(check_sector(s));
  if (spin != 0 && spin != 1) return invalid("spin must be 0 or 1");
  const SpinTables& T = spin == 0 ? s->up : s->dw;
  const int64_t D = T.D;
  if (map) EDX_HIP(hipMemcpy(map, T.map, D * sizeof(uint32_t), hipMemcpyDeviceToHost));
  if (diag_e) EDX_HIP(hipMemcpy(diag_e, T.e64, D * sizeof(double), hipMemcpyDeviceToHost));
  if (diag_p) EDX_HIP(hipMemcpy(diag_p, T.pat, D, hipMemcpyDeviceToHost));
  if (hop_off || hop_col || hop_sign || hop_amp) {
    std::vector<uint32_t> ell((size_t)T.wpad * D);
    EDX_HIP(hipMemcpy(ell.data(), T.hop, ell.size() * sizeof(uint32_t), hipMemcpyDeviceToHost));
    int64_t pos = 0;
    std::vector<std::pair<uint32_t, uint32_t>> row;
    for (int64_t i = 0; i < D; ++i) {
      if (hop_off) hop_off[i] = pos;
      row.clear();
      for (int k = 0; k < T.wpad; ++k) {
        const uint32_t e = ell[(size_t)i * T.wpad + k];
        if (((e >> kAmpShift) & 0x7Fu) == kPadPair) continue;
        row.emplace_back(e & kColMask, e);
      }
      std::sort(row.begin(), row.end());
      for (auto& ce : row) {
        if (hop_col) hop_col[pos] = (int32_t)ce.first;
        if (hop_sign) hop_sign[pos] = (ce.second >> 31) ? -1 : 1;
        if (hop_amp) hop_amp[pos] = s->amp_host[ce.second >> kAmpShift];
        ++pos;
      }
    }
    if (hop_off) hop_off[D] = pos;
  }
  return EDX_OK;
}

edx_status edx_sector_get_rank(const edx_sector* s, int32_t spin, int32_t* rank) {
  EDX_TRY(check_sector(s));
  if (spin != 0 && spin != 1) return invalid("spin must be 0 or 1");
  if (!rank) return invalid("rank is NULL");
  const SpinTables& T = spin == 0 ? s->up : s->dw;
  const size_t total = size_t(1) << s->model.ns;
  EDX_HIP(hipMemcpy(rank, T.rank, total * sizeof(int32_t), hipMemcpyDeviceToHost));
  return EDX_OK;
}

edx_status edx_hv(const edx_sector* s, edx_vtype vtype, const void* v, void* w, int64_t ld,
                  void* stream) {
  EDX_TRY(check_sector(s));
  if (!valid_vtype(vtype)) return invalid("vtype must be EDX_F64 or EDX_F32");
  if (!v || !w) return invalid("v or w is NULL");
  if (ld == 0) ld = s->dup;
  if (ld < s->dup) return invalid("ld must be 0 (dense) or >= D_up");
  const size_t bytes = (size_t)(ld * s->ddw * s->dph) * vbytes(vtype);
  const char* pv = static_cast<const char*>(v);
  const char* pw = static_cast<const char*>(w);
  if (pv < pw + bytes && pw < pv + bytes) return invalid("v and w overlap");
  return hv_launch(s, vtype, v, w, ld, nullptr, nullptr, static_cast<hipStream_t>(stream));
}

size_t edx_hv_multi_workspace_bytes(const edx_sector* const* secs, int32_t k, int32_t vtype) {
  if (!secs || !secs[0] || !valid_vtype(vtype) || (k != 1 && k != 2 && k != 4 && k != 8)) return 0;
  return multi_hv_workspace_bytes(secs[0], k, vtype);
}

edx_status edx_hv_multi(const edx_sector* const* secs, int32_t k, edx_vtype vtype, const void* v,
                        void* w, void* ws, size_t ws_bytes, void* stream) {
  if (!secs || !v || !w || !ws) return invalid("secs, v, w and ws must be non-NULL");
  if (!valid_vtype(vtype)) return invalid("vtype must be EDX_F64 or EDX_F32");
  if (k != 1 && k != 2 && k != 4 && k != 8) return invalid("k must be 1, 2, 4 or 8");
  for (int b = 0; b < k; ++b) EDX_TRY(check_sector(secs[b]));
  const size_t bytes = (size_t)(secs[0]->vlen * k) * vbytes(vtype);
  const char* pv = static_cast<const char*>(v);
  const char* pw = static_cast<const char*>(w);
  if (pv < pw + bytes && pw < pv + bytes) return invalid("v and w overlap");
  return multi_hv(secs, k, vtype, v, w, ws, ws_bytes, static_cast<hipStream_t>(stream));
}

edx_status edx_hv_block(const edx_sector* s, edx_vtype vtype, int32_t part, const void* v,
                        void* w, int64_t ld, int64_t c0, int64_t c1, void* stream) {
  EDX_TRY(check_sector(s));
  if (!valid_vtype(vtype)) return invalid("vtype must be EDX_F64 or EDX_F32");
  if (!v || !w) return invalid("v or w is NULL");
  if (part != 0 && part != 1) return invalid("part must be 0 or 1");
  if (s->nd) {
    set_error("hv_block: spin exchange / pair hopping couple both spins (no column-local form)");
    return EDX_E_UNSUPPORTED;
  }
  const int64_t rows = part == 0 ? s->dup : s->ddw;
  const int64_t cols = part == 0 ? s->ddw : s->dup;
  if (ld < rows) return invalid("ld below the column length");
  if (c0 < 0 || c1 > cols || c0 >= c1) return invalid("column range outside [0, ncols)");
  const size_t bytes = (size_t)(ld * cols) * vbytes(vtype);
  const char* pv = static_cast<const char*>(v);
  const char* pw = static_cast<const char*>(w);
  if (pv < pw + bytes && pw < pv + bytes) return invalid("v and w overlap");
  return hv_block_launch(s, vtype, part, v, w, ld, c0, c1, static_cast<hipStream_t>(stream));
}

edx_status edx_transpose(edx_vtype vtype, const void* src, int64_t rows, int64_t cols,
                         int64_t lds, void* dst, int64_t ldd, int32_t add, void* stream) {
  if (!valid_vtype(vtype)) return invalid("vtype must be EDX_F64 or EDX_F32");
  if (!src || !dst) return invalid("src or dst is NULL");
  if (rows < 0 || cols < 0 || lds < rows || ldd < cols) return invalid("bad shape or stride");
  if (add != 0 && add != 1) return invalid("add must be 0 or 1");
  return k_transpose(vtype, src, rows, cols, lds, dst, ldd, add, static_cast<hipStream_t>(stream));
}

edx_status edx_hv_get_plan(const edx_sector* s, edx_vtype vtype, edx_hv_plan* plan) {
  if (!s || !plan) return invalid("sector or plan is NULL");
  if (!valid_vtype(vtype)) return invalid("vtype must be EDX_F64 or EDX_F32");
  const HvPlan p = hv_plan(s, vtype);
  plan->mode = p.mode;
  plan->col_cols = p.col_cols;
  plan->col_threads = p.col_threads;
  plan->row_rows = p.row_rows;
  plan->row_cols = p.row_cols;
  plan->col_order = p.col_order;
  return EDX_OK;
}

edx_status edx_hv_set_plan(edx_sector* s, edx_vtype vtype, const edx_hv_plan* plan) {
  if (!s || !plan) return invalid("sector or plan is NULL");
  if (!valid_vtype(vtype)) return invalid("vtype must be EDX_F64 or EDX_F32");
  HvPlan p;
  p.mode = plan->mode;
  p.col_cols = plan->col_cols;
  p.col_threads = plan->col_threads;
  p.row_rows = plan->row_rows;
  p.row_cols = plan->row_cols;
  p.col_order = plan->col_order;
  EDX_TRY(hv_validate(s, vtype, &p));
  const int k = vtype == EDX_F32 ? 1 : 0;
  s->plan[k] = p;
  s->plan_set[k] = true;
  return EDX_OK;
}

edx_status edx_autotune_hv(edx_sector* s, edx_vtype vtype, const void* v, void* w, int64_t ld,
                           int32_t reps, void* stream, edx_hv_plan* best, double* best_us) {
  EDX_TRY(check_sector(s));
  if (!valid_vtype(vtype)) return invalid("vtype must be EDX_F64 or EDX_F32");
  if (!v || !w) return invalid("v or w is NULL");
  if (ld == 0) ld = s->dup;
  if (ld < s->dup) return invalid("ld must be 0 (dense) or >= D_up");
  HvPlan bp;
  EDX_TRY(hv_autotune(s, vtype, v, w, ld, std::max(1, (int)reps),
                      static_cast<hipStream_t>(stream), &bp, best_us));
  if (best) {
    best->mode = bp.mode;
    best->col_cols = bp.col_cols;
    best->col_threads = bp.col_threads;
    best->row_rows = bp.row_rows;
    best->row_cols = bp.row_cols;
    best->col_order = bp.col_order;
  }
  return EDX_OK;
}

void edx_lanczos_default_opts(edx_lanczos_opts* o) {
  if (!o) return;
  o->niter = 512;
  o->vtype = EDX_F64;
  o->reorth = 0;
  o->check_every = 8;
  o->tol = 1e-12;
  o->rtol = 0.0;
  o->seed = 1234567;
  o->degen_check = 1;
  o->pad_ = 0;
  o->start = nullptr;
}

size_t edx_workspace_bytes(const edx_sector* s, int32_t what, int32_t vtype, int32_t n) {
  if (!s || !valid_vtype(vtype) || n < 1) return 0;
  if (what == EDX_WS_LANCZOS) return lanczos_workspace_bytes(s, vtype, n, 0);
  if (what == EDX_WS_GREEN) return green_workspace_bytes(s, vtype, n);
  if (what == 2) return lanczos_workspace_bytes(s, vtype, n, 2);   // full re-orthogonalisation
  if (what == EDX_WS_CHI) return chi_workspace_bytes(s, vtype, n);
  if (what == EDX_WS_PAIR) return pair_workspace_bytes(s, vtype, n);
  return 0;
}

edx_status edx_lanczos_ground_state(const edx_sector* s, const edx_lanczos_opts* opts, void* ws,
                                    size_t ws_bytes, double* e0, void* psi0,
                                    edx_lanczos_report* rep, void* stream) {
  EDX_TRY(check_sector(s));
  if (!opts || !e0 || !ws) return invalid("opts, e0 and ws must be non-NULL");
  if (!valid_vtype(opts->vtype)) return invalid("vtype must be EDX_F64 or EDX_F32");
  if (opts->niter < 1 || opts->niter > 4096) return invalid("niter must be in [1, 4096]");
  if (opts->reorth < 0 || opts->reorth > 3) return invalid("reorth must be 0, 1, 2 or 3");
  if (!(opts->tol >= 0.0) || !(opts->rtol >= 0.0)) return invalid("tol/rtol must be >= 0");
  return lanczos_ground_state_impl(s, opts, ws, ws_bytes, e0, psi0, rep,
                                   static_cast<hipStream_t>(stream));
}

edx_status edx_lanczos_ground_state_static(const edx_sector* s, const edx_lanczos_opts* opts,
                                           double* e0, void* psi0, edx_lanczos_report* rep,
                                           void* stream) {
  EDX_TRY(check_sector(s));
  if (!opts || !e0) return invalid("opts and e0 must be non-NULL");
  if (!valid_vtype(opts->vtype)) return invalid("vtype must be EDX_F64 or EDX_F32");
  if (opts->niter < 1 || opts->niter > 4096) return invalid("niter must be in [1, 4096]");
  if (opts->reorth < 0 || opts->reorth > 3) return invalid("reorth must be 0, 1, 2 or 3");
  if (!(opts->tol >= 0.0) || !(opts->rtol >= 0.0)) return invalid("tol/rtol must be >= 0");
  return lanczos_ground_state_static(s, opts, e0, psi0, rep, static_cast<hipStream_t>(stream));
}

size_t edx_lowest_workspace_bytes(const edx_sector* s, int32_t vtype, int32_t niter, int32_t k) {
  if (!s || !valid_vtype(vtype) || niter < 1 || k < 1 || k > EDX_MAX_STATES) return 0;
  return lowest_workspace_bytes(s, vtype, niter, k);
}

edx_status edx_lanczos_lowest(const edx_sector* s, int32_t k, const edx_lanczos_opts* opts,
                              int32_t verify, void* ws, size_t ws_bytes, double* e, void* psi,
                              edx_lowest_report* rep, void* stream) {
  EDX_TRY(check_sector(s));
  if (!opts || !e || !ws) return invalid("opts, e and ws must be non-NULL");
  if (k < 1 || k > EDX_MAX_STATES) return invalid("k must be in [1, 64]");
  if (!valid_vtype(opts->vtype)) return invalid("vtype must be EDX_F64 or EDX_F32");
  if (opts->niter < 1 || opts->niter > 4096) return invalid("niter must be in [1, 4096]");
  if (!(opts->tol >= 0.0) || !(opts->rtol >= 0.0) || !(opts->tol > 0.0 || opts->rtol > 0.0))
    return invalid("tol/rtol must be >= 0, one of them > 0");
  return lowest_states_impl(s, k, opts, verify, ws, ws_bytes, e, psi, rep,
                            static_cast<hipStream_t>(stream));
}

edx_status edx_tridiag_spectrum(const double* alpha, const double* beta, int32_t m,
                                double* theta, double* weight) {
  if (m < 1 || !alpha || !theta || !weight || (m > 1 && !beta))
    return invalid("alpha, beta, theta, weight must be non-NULL and m >= 1");
  if (!tridiag_spectrum(alpha, beta, m, theta, weight)) {
    set_error("tridiag_spectrum: QR iteration did not converge");
    return EDX_E_NOCONV;
  }
  return EDX_OK;
}

edx_status edx_chi(const edx_sector* s, const void* psi0, double e0, const double* cu,
                   const double* cd, const edx_gf_opts* opts, void* ws, size_t ws_bytes,
                   double* chi_host, edx_chi_report* rep, void* stream) {
  EDX_TRY(check_sector(s));
  if (!psi0 || !cu || !cd || !opts || !ws || !chi_host)
    return invalid("psi0, cu, cd, opts, ws and chi_host must be non-NULL");
  if (!valid_vtype(opts->vtype)) return invalid("vtype must be EDX_F64 or EDX_F32");
  if (opts->ngf > 4096) return invalid("ngf must be <= 4096");
  DiagCoef c{};
  for (int a = 0; a < s->model.norb; ++a) {
    if (!std::isfinite(cu[a]) || !std::isfinite(cd[a])) return invalid("cu/cd must be finite");
    c.up[a] = cu[a];
    c.dw[a] = cd[a];
  }
  return chi_impl(s, psi0, e0, c, opts, ws, ws_bytes, chi_host, rep,
                  static_cast<hipStream_t>(stream));
}

edx_status edx_chi_exciton(const edx_sector* s, const void* psi0, double e0, int32_t a,
                           int32_t b, const edx_gf_opts* opts, void* ws, size_t ws_bytes,
                           double* chi_host, edx_chi_report* rep, void* stream) {
  EDX_TRY(check_sector(s));
  if (!psi0 || !opts || !ws || !chi_host) return invalid("psi0, opts, ws and chi_host must be non-NULL");
  if (!valid_vtype(opts->vtype)) return invalid("vtype must be EDX_F64 or EDX_F32");
  if (opts->ngf > 4096) return invalid("ngf must be <= 4096");
  if (a < 0 || b < 0 || a >= s->model.norb || b >= s->model.norb || a == b)
    return invalid("a and b must be two different orbitals");
  if (s->orb || s->dph > 1) {
    set_error("chi_exciton: needs a total-N sector without phonons");
    return EDX_E_UNSUPPORTED;
  }
  DiagCoef c{};
  return chi_impl(s, psi0, e0, c, opts, ws, ws_bytes, chi_host, rep,
                  static_cast<hipStream_t>(stream), 1, std::min(a, b), std::max(a, b));
}

edx_status edx_chi_pair(const edx_sector* gs, const void* psi0, double e0, int32_t a,
                        const edx_gf_opts* opts, void* ws, size_t ws_bytes, double* chi_host,
                        edx_gf_report* rep, void* stream) {
  EDX_TRY(check_sector(gs));
  if (!psi0 || !opts || !ws || !chi_host) return invalid("psi0, opts, ws and chi_host must be non-NULL");
  if (!valid_vtype(opts->vtype)) return invalid("vtype must be EDX_F64 or EDX_F32");
  if (opts->ngf > 4096) return invalid("ngf must be <= 4096");
  if (a < 0 || a >= gs->model.norb) return invalid("orbital out of range");
  if (gs->dph > 1) {
    set_error("chi_pair: sectors with phonons are not supported");
    return EDX_E_UNSUPPORTED;
  }
  return pair_impl(gs, psi0, e0, a, opts, ws, ws_bytes, chi_host, rep,
                   static_cast<hipStream_t>(stream));
}

edx_status edx_green_cf(const edx_sector* gs, const void* psi0, double e0, int32_t orb,
                        int32_t spin, const edx_gf_opts* opts, void* ws, size_t ws_bytes,
                        double* g_host, edx_gf_report* rep, void* stream) {
  EDX_TRY(check_sector(gs));
  if (!opts || !psi0 || !ws || !g_host) return invalid("opts, psi0, ws and g_host must be non-NULL");
  if (!valid_vtype(opts->vtype)) return invalid("vtype must be EDX_F64 or EDX_F32");
  if (orb < 0 || orb >= gs->model.norb) return invalid("orb out of range");
  if (spin != 0 && spin != 1) return invalid("spin must be 0 or 1");
  if (opts->ngf > 4096) return invalid("ngf must be <= 4096");
  return green_cf_impl(gs, psi0, e0, orb, spin, opts, ws, ws_bytes, g_host, rep,
                       static_cast<hipStream_t>(stream));
}

size_t edx_batch_workspace_bytes(const edx_sector* const* sectors, int32_t n, int32_t vtype,
                                 int32_t lane_wgs, int64_t wide_min_dim) {
  if (!sectors || n < 1 || !valid_vtype(vtype) || lane_wgs < 1) return 0;
  for (int i = 0; i < n; ++i)
    if (!sectors[i]) return 0;
  return batch_workspace_bytes(sectors, n, vtype, lane_wgs, wide_min_dim);
}

static edx_status check_batch(const edx_sector* const* sectors, int32_t n,
                              const edx_lanczos_opts* opts) {
  if (!sectors || n < 1 || !opts) return invalid("sectors, n >= 1 and opts are required");
  if (!valid_vtype(opts->vtype)) return invalid("vtype must be EDX_F64 or EDX_F32");
  if (opts->reorth != 0) return invalid("the batched solver runs plain Lanczos (reorth = 0)");
  if (opts->niter < 1 || opts->niter > 2048) return invalid("niter must be in [1, 2048]");
  for (int i = 0; i < n; ++i) EDX_TRY(check_sector(sectors[i]));
  return EDX_OK;
}

edx_status edx_batch_ground_state(const edx_sector* const* sectors, int32_t n,
                                  const edx_lanczos_opts* opts, const edx_batch_tiles* tiles,
                                  void* ws, size_t ws_bytes, edx_batch_result* results,
                                  double* elapsed_ms, void* stream) {
  EDX_TRY(check_batch(sectors, n, opts));
  if (!ws || !results) return invalid("ws and results must be non-NULL");
  const int L = tiles ? tiles->lane_wgs : 32;
  if (L != 8 && L != 16 && L != 32) return invalid("lane_wgs must be 8, 16 or 32");
  const int mk = tiles ? tiles->multi_k : 0;
  if (mk < 0 || mk > 8) return invalid("tiles.multi_k must be in [0, 8]");
  return batch_run(sectors, n, opts, tiles ? tiles->ccols : nullptr,
                   tiles ? tiles->rcols : nullptr, L, tiles ? tiles->wide_min_dim : 0, mk, ws,
                   ws_bytes, results, static_cast<hipStream_t>(stream), elapsed_ms);
}

edx_status edx_batch_autotune(const edx_sector* const* sectors, int32_t n,
                              const edx_lanczos_opts* opts, void* ws, size_t ws_bytes,
                              int32_t* ccols, int32_t* rcols, int32_t* lane_wgs,
                              int64_t* wide_min_dim, void* stream) {
  EDX_TRY(check_batch(sectors, n, opts));
  if (!ws || !ccols || !rcols || !lane_wgs || !wide_min_dim)
    return invalid("ws and outputs must be non-NULL");
  return batch_autotune(sectors, n, opts, ws, ws_bytes, ccols, rcols, lane_wgs, wide_min_dim,
                        static_cast<hipStream_t>(stream));
}

const char* edx_status_str(edx_status st) {
  switch (st) {
    case EDX_OK: return "EDX_OK";
    case EDX_E_INVALID: return "EDX_E_INVALID";
    case EDX_E_NOMEM: return "EDX_E_NOMEM";
    case EDX_E_DEVICE: return "EDX_E_DEVICE";
    case EDX_E_NOCONV: return "EDX_E_NOCONV";
    case EDX_E_DEGENERATE: return "EDX_E_DEGENERATE";
    case EDX_E_UNSUPPORTED: return "EDX_E_UNSUPPORTED";
    case EDX_PENDING: return "EDX_PENDING";
  }
  return "EDX_E_UNKNOWN";
}

const char* edx_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
