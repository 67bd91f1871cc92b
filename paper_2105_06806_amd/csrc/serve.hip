// Continuous-batching request server (host runtime).
//
// Requests (model, sector) arrive at any time and each asks for the ground
// state and, optionally, the impurity Green's function.  The server holds one
// device arena of a fixed size (allocated once at creation) and `max_slots`
// worker threads, each with its own HIP stream.  Admission is by device
// footprint: a request is admitted when a worker is free and its workspace
// (Lanczos vectors, psi0, Green vectors) fits in the arena; the smallest
// pending request that fits goes first (small sectors are quick, so they do
// not wait behind large ones), at most kLargeCap requests of `kLargeBytes`
// or more run at once, and a request passed over `kMaxSkips` times blocks
// further passing until it is admitted (no starvation).  Admitted requests
// run concurrently on their streams, so their kernels overlap on the device;
// a request that arrives while others run is admitted as soon as a slot and
// memory free up.  Every request runs the same kernels with the same launch
// shapes as the plain API, whatever else is running, so its result is
// bitwise the same alone and in the mix.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "edx_internal.h"

namespace edx {

namespace {

constexpr int kMaxSkips = 8;
constexpr size_t kLargeBytes = size_t(1) << 30;   // a "large" request's footprint
// Large requests in flight at once.  They are bandwidth-bound, so running them
// one at a time loses no throughput, and each finishes sooner: on the
// 1000-request Ns 10..16 stream, one instead of half the slots gave p99 2.28
// vs 2.99 s at half the one-at-a-time capacity and 15.9 vs 18.3 s at the
// full capacity (p50 0.058 vs 0.062 s and 0.088 vs 0.342 s, the same
// throughput).
constexpr int kLargeCap = 1;
constexpr size_t kAlign = 256;

double now_s() {
  using C = std::chrono::steady_clock;
  static const C::time_point t0 = C::now();
  return std::chrono::duration<double>(C::now() - t0).count();
}

int64_t binom(int n, int k) {
  if (k < 0 || k > n) return 0;
  int64_t r = 1;
  for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
  return r;
}

// First-fit allocator over one device range; offsets aligned to 256 bytes.
class Arena {
 public:
  void init(char* base, size_t size) {
    base_ = base;
    free_.clear();
    free_[0] = size;
  }
  char* alloc(size_t bytes) {
    bytes = align_up(bytes, kAlign);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        const size_t off = it->first;
        const size_t rest = it->second - bytes;
        free_.erase(it);
        if (rest) free_[off + bytes] = rest;
        return base_ + off;
      }
    }
    return nullptr;
  }
  void release(char* p, size_t bytes) {
    bytes = align_up(bytes, kAlign);
    size_t off = (size_t)(p - base_);
    auto next = free_.lower_bound(off);
    if (next != free_.end() && off + bytes == next->first) {
      bytes += next->second;
      next = free_.erase(next);
    }
    if (next != free_.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == off) {
        prev->second += bytes;
        return;
      }
    }
    free_[off] = bytes;
  }
  size_t largest() const {
    size_t m = 0;
    for (auto& kv : free_) m = std::max(m, kv.second);
    return m;
  }

 private:
  char* base_ = nullptr;
  std::map<size_t, size_t> free_;
};

// Bump allocator over the table region of one request's block.
struct Bump {
  char* base = nullptr;
  size_t off = 0, cap = 0;
  static void* alloc(void* ctx, size_t bytes) {
    Bump* b = static_cast<Bump*>(ctx);
    const size_t o = align_up(b->off, kAlign);
    if (o + bytes > b->cap) return nullptr;
    b->off = o + bytes;
    return b->base + o;
  }
  static void release(void*, void*) {}
};

struct Request {
  int64_t ticket = 0;
  Model model;
  int nup = 0, ndw = 0;
  size_t footprint = 0;
  size_t table_bytes = 0;
  int skips = 0;
  double t_submit = 0, t_start = 0, t_done = 0;
  edx_status status = EDX_OK;
  double e0 = 0, wp = 0, wh = 0;
  int iters = 0;
  std::vector<double> g;
  bool done = false;
};

}  // namespace
}  // namespace edx

struct edx_server {
  edx_server_opts opts;
  char* dev_base = nullptr;
  edx::Arena arena;
  std::mutex mu;
  std::condition_variable cv_work;   // workers wait for admissible requests
  std::condition_variable cv_done;   // pollers wait for completions
  std::deque<edx::Request*> pending;
  std::map<int64_t, std::unique_ptr<edx::Request>> all;
  std::vector<std::thread> workers;
  std::vector<hipStream_t> streams;
  int64_t next_ticket = 1;
  int busy = 0;
  int large = 0;      // running requests with footprint >= kLargeBytes
  bool stop = false;
  int device = 0;
  std::atomic<int64_t> completed{0};
};

namespace edx {
namespace {

// Device bytes a request needs from the arena: Lanczos workspace, psi0 and
// the Green's-function workspace, from the sector dimensions.
size_t estimate_tables(const edx_server_opts& o, const Model& m, int nup, int ndw) {
  size_t b = sector_table_bytes(m.ns, nup, ndw);
  if (o.ngf > 0) {
    if (nup + 1 <= m.ns) b += sector_table_bytes(m.ns, nup + 1, ndw);
    if (nup - 1 >= 0) b += sector_table_bytes(m.ns, nup - 1, ndw);
  }
  return align_up(b, kAlign);
}

size_t estimate_footprint(const edx_server_opts& o, const Model& m, int nup, int ndw) {
  const size_t vb = vbytes(o.vtype);
  const int ns = m.ns;
  const int64_t dup = binom(ns, nup), ddw = binom(ns, ndw), dim = dup * ddw;
  const int niter = o.lanczos.niter;
  auto lanc = [&](int64_t d, int64_t cols, int n) {
    return align_up((size_t)d * vb) * 3 +
           align_up(sizeof(double) * (size_t)std::max<int64_t>(2 * kMaxPartials,
                                                               cols + 8 + kNdMaxBlocks)) +
           8 * align_up(sizeof(double) * (size_t)(n + 2)) + 4096;
  };
  // Krylov vectors use the padded column stride; psi0 is accumulated in that
  // layout (one more vector when it differs) and returned densely
  const int64_t ld = vec_ld(dup), vlen = ld * ddw;
  size_t bytes = lanc(vlen, ddw, niter) + (ld != dup ? align_up((size_t)vlen * vb) : 0) +
                 align_up((size_t)dim * vb);
  if (o.ngf > 0) {
    int64_t dmax = 1;
    for (int d : {-1, 1}) {
      dmax = std::max(dmax, vec_ld(binom(ns, nup + d)) * ddw);
      dmax = std::max(dmax, ld * binom(ns, ndw + d));
    }
    const int64_t cmax = std::max({binom(ns, ndw - 1), ddw, binom(ns, ndw + 1)});
    bytes += lanc(dmax, cmax, o.ngf) + sizeof(double) * (2 * 65536 + 4 * (o.ngf + 1)) + 1024;
  }
  return bytes + 3 * kAlign + estimate_tables(o, m, nup, ndw);
}

void worker_main(edx_server* S, int slot) {
  (void)hipSetDevice(S->device);
  hipStream_t st = S->streams[slot];
  for (;;) {
    Request* R = nullptr;
    char* mem = nullptr;
    {
      std::unique_lock<std::mutex> lk(S->mu);
      for (;;) {
        if (S->stop) return;
        // admission, smallest footprint first (the footprint grows with the
        // sector dimension, so with the work): among the admissible pending
        // requests -- a large one (footprint >= kLargeBytes) only while fewer
        // than kLargeCap run, so small requests always find a slot and the
        // large ones do not share the bandwidth with each other --
        // the smallest that fits is taken, and every older admissible request
        // it passes counts a skip; the oldest admissible request passed over
        // kMaxSkips times goes next, waiting for memory if need be (nothing
        // passes it), so none starves
        const int large_cap = std::min(kLargeCap, S->opts.max_slots);
        auto admissible = [&](const Request* q) {
          return q->footprint < kLargeBytes || S->large < large_cap;
        };
        Request* due = nullptr;
        for (Request* q : S->pending)
          if (admissible(q) && q->skips >= kMaxSkips) {
            due = q;
            break;
          }
        if (due) {
          mem = S->arena.alloc(due->footprint);
          if (mem) R = due;
        } else {
          std::vector<Request*> bysize;
          for (Request* q : S->pending)
            if (admissible(q)) bysize.push_back(q);
          std::stable_sort(bysize.begin(), bysize.end(), [](const Request* x, const Request* y) {
            return x->footprint < y->footprint;
          });
          for (Request* q : bysize) {
            mem = S->arena.alloc(q->footprint);
            if (mem) {
              R = q;
              break;
            }
          }
        }
        if (R) {
          for (auto it = S->pending.begin(); it != S->pending.end();) {
            if (*it == R) {
              it = S->pending.erase(it);
              break;
            }
            if (admissible(*it)) ++(*it)->skips;   // older than R and passed over
            ++it;
          }
          if (R->footprint >= kLargeBytes) ++S->large;
          break;
        }
        S->cv_work.wait(lk);
      }
      ++S->busy;
      R->t_start = now_s();
    }
    // run: tables, ground state with psi0, Green's function
    const edx_server_opts& o = S->opts;
    edx_sector* sec = nullptr;
    // block layout: [tables of the sector and its Green's-function neighbours |
    //                Lanczos workspace | psi0 | Green workspace]
    Bump bump;
    bump.base = mem;
    bump.cap = R->table_bytes;
    Allocator al;
    al.alloc = &Bump::alloc;
    al.release = &Bump::release;
    al.ctx = &bump;
    edx_status st2 = build_sector_impl(R->model, R->nup, R->ndw, st, &sec, &al);
    if (st2 == EDX_OK) {
      const size_t vb = vbytes(o.vtype);
      const size_t lw = lanczos_workspace_bytes(sec, o.vtype, o.lanczos.niter, 0);
      const size_t pb = align_up((size_t)sec->dim * vb);
      const size_t gw = o.ngf > 0 ? green_workspace_bytes(sec, o.vtype, o.ngf) : 0;
      if (R->table_bytes + align_up(lw) + pb + gw > R->footprint) {
        st2 = EDX_E_NOMEM;
        set_error("serve: footprint estimate below the exact workspace");
      } else {
        char* ws = mem + R->table_bytes;
        char* psi = ws + align_up(lw);
        char* gws = psi + pb;
        edx_lanczos_opts lo = o.lanczos;
        lo.vtype = o.vtype;
        lo.reorth = 0;
        lo.start = nullptr;
        edx_lanczos_report rep{};
        double e0 = 0;
        st2 = lanczos_ground_state_impl(sec, &lo, ws, lw, &e0, psi, &rep, st);
        R->e0 = e0;
        R->iters = rep.iters;
        if ((st2 == EDX_OK || st2 == EDX_E_DEGENERATE) && o.ngf > 0) {
          edx_gf_opts go{o.ngf, o.lmats, o.vtype, 0, o.beta};
          edx_gf_report gr{};
          R->g.assign(2 * (size_t)o.lmats, 0.0);
          const edx_status sg = green_cf_impl(sec, psi, e0, 0, 0, &go, gws, gw, R->g.data(), &gr, st);
          R->wp = gr.wp;
          R->wh = gr.wh;
          if (sg != EDX_OK) st2 = sg;
        }
      }
      destroy_sector(sec);
    }
    {
      std::lock_guard<std::mutex> lk(S->mu);
      S->arena.release(mem, R->footprint);
      if (R->footprint >= kLargeBytes) --S->large;
      R->status = st2;
      R->t_done = now_s();
      R->done = true;
      --S->busy;
      S->completed++;
    }
    S->cv_work.notify_all();
    S->cv_done.notify_all();
  }
}

}  // namespace
}  // namespace edx

using namespace edx;

extern "C" {

void edx_server_default_opts(edx_server_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->hbm_budget = (size_t)8 << 30;
  o->max_slots = 8;
  o->vtype = EDX_F32;
  o->ngf = 200;
  o->lmats = 1024;
  o->beta = 200.0;
  edx_lanczos_default_opts(&o->lanczos);
  o->lanczos.vtype = EDX_F32;
}

edx_status edx_server_create(const edx_server_opts* opts, edx_server** out) {
  if (!opts || !out) {
    set_error("opts and out are required");
    return EDX_E_INVALID;
  }
  *out = nullptr;
  if (opts->max_slots < 1 || opts->max_slots > 64 || opts->hbm_budget < ((size_t)1 << 20) ||
      (opts->vtype != EDX_F32 && opts->vtype != EDX_F64) || opts->ngf < 0 ||
      (opts->ngf > 0 && (opts->lmats < 1 || opts->lmats > 65536 || !(opts->beta > 0))) ||
      opts->lanczos.niter < 1 || opts->lanczos.niter > 4096) {
    set_error("server: invalid options");
    return EDX_E_INVALID;
  }
  std::unique_ptr<edx_server> S(new edx_server());
  S->opts = *opts;
  EDX_HIP(hipGetDevice(&S->device));
  EDX_HIP(hipMalloc(&S->dev_base, opts->hbm_budget));
  S->arena.init(S->dev_base, opts->hbm_budget);
  S->streams.resize(opts->max_slots);
  for (auto& st : S->streams) EDX_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
  for (int i = 0; i < opts->max_slots; ++i) S->workers.emplace_back(worker_main, S.get(), i);
  *out = S.release();
  return EDX_OK;
}

edx_status edx_server_submit(edx_server* S, const edx_model* model, int32_t nup, int32_t ndw,
                             int64_t* ticket) {
  if (!S || !model || !ticket) {
    set_error("server, model and ticket are required");
    return EDX_E_INVALID;
  }
  auto R = std::make_unique<Request>();
  // reuse the builder's validation through a throwaway copy of the checks
  const int ns = model->norb * (model->nbath + 1);
  if (model->norb < 1 || model->norb > kMaxNorb || model->nbath < 0 || ns > kMaxNs ||
      !model->eps_imp || (model->nbath > 0 && (!model->eps_bath || !model->vhyb)) || nup < 0 ||
      ndw < 0 || nup > ns || ndw > ns) {
    set_error("server: invalid model or sector");
    return EDX_E_INVALID;
  }
  Model& m = R->model;
  m.norb = model->norb;
  m.nbath = model->nbath;
  m.ns = ns;
  m.eps_imp.assign(model->eps_imp, model->eps_imp + m.norb);
  m.eps_bath.assign(model->eps_bath, model->eps_bath + m.norb * m.nbath);
  m.vhyb.assign(model->vhyb, model->vhyb + m.norb * m.nbath);
  m.U = model->U;
  m.Ust = model->Ust;
  m.Jh = model->Jh;
  m.xmu = model->xmu;
  m.Jx = model->Jx;
  m.Jp = model->Jp;
  if (!std::isfinite(m.Jx) || !std::isfinite(m.Jp)) {
    set_error("server: non-finite interaction parameter");
    return EDX_E_INVALID;
  }
  if (model->nph != 0) {
    set_error("server: models with phonons are not served (use the direct entry points)");
    return EDX_E_UNSUPPORTED;
  }
  R->nup = nup;
  R->ndw = ndw;
  R->footprint = estimate_footprint(S->opts, m, nup, ndw);
  R->table_bytes = estimate_tables(S->opts, m, nup, ndw);
  if (R->footprint > S->opts.hbm_budget) {
    set_error("server: request larger than the whole arena");
    return EDX_E_NOMEM;
  }
  {
    std::lock_guard<std::mutex> lk(S->mu);
    R->ticket = S->next_ticket++;
    R->t_submit = now_s();
    *ticket = R->ticket;
    S->pending.push_back(R.get());
    S->all[R->ticket] = std::move(R);
  }
  S->cv_work.notify_all();
  return EDX_OK;
}

edx_status edx_server_poll(edx_server* S, int64_t ticket, int32_t wait, edx_server_result* res,
                           double* g_out) {
  if (!S || !res) {
    set_error("server and result are required");
    return EDX_E_INVALID;
  }
  std::unique_lock<std::mutex> lk(S->mu);
  auto it = S->all.find(ticket);
  if (it == S->all.end()) {
    set_error("server: unknown ticket");
    return EDX_E_INVALID;
  }
  Request* R = it->second.get();
  if (!R->done) {
    if (!wait) return EDX_PENDING;
    S->cv_done.wait(lk, [&] { return R->done; });
  }
  res->ticket = R->ticket;
  res->status = R->status;
  res->iters = R->iters;
  res->e0 = R->e0;
  res->wp = R->wp;
  res->wh = R->wh;
  res->t_submit = R->t_submit;
  res->t_start = R->t_start;
  res->t_done = R->t_done;
  res->footprint = R->footprint;
  if (g_out && !R->g.empty()) std::memcpy(g_out, R->g.data(), R->g.size() * sizeof(double));
  S->all.erase(it);
  return EDX_OK;
}

edx_status edx_server_stats(edx_server* S, int32_t* pending, int32_t* running,
                            int64_t* completed, size_t* largest_free) {
  if (!S) {
    set_error("server is NULL");
    return EDX_E_INVALID;
  }
  std::lock_guard<std::mutex> lk(S->mu);
  if (pending) *pending = (int32_t)S->pending.size();
  if (running) *running = S->busy;
  if (completed) *completed = S->completed.load();
  if (largest_free) *largest_free = S->arena.largest();
  return EDX_OK;
}

double edx_server_clock(void) { return now_s(); }

void edx_server_destroy(edx_server* S) {
  if (!S) return;
  {
    std::unique_lock<std::mutex> lk(S->mu);
    // let admitted work finish; drop what was never admitted
    S->cv_done.wait(lk, [&] { return S->busy == 0; });
    S->stop = true;
  }
  S->cv_work.notify_all();
  for (auto& t : S->workers) t.join();
  for (auto& st : S->streams) (void)hipStreamDestroy(st);
  (void)hipFree(S->dev_base);
  delete S;
}

}  // extern "C"
