// Internal declarations shared by the translation units of libedx.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/edx.h"

namespace edx {

constexpr int kMaxNs = 24;
constexpr int kMaxNorb = 3;
constexpr int kMaxPh = 63;                   // phonon cutoff N_ph (D_ph <= 64)
constexpr uint32_t kColMask = 0x00FFFFFFu;   // hop entry: bits 0..23 column
constexpr int kAmpShift = 24;                // bits 24..30 pair, bit 31 sign
constexpr uint32_t kPadPair = 0x7Fu;         // pair index of padding entries
constexpr int kAmpTable = 256;               // signed amplitude per (pair, sign)
constexpr int kMaxPartials = 2048;           // partial sums per reduction
constexpr int kReduceSlots = 8;              // dots reduced by one kernel
constexpr int kNdMaxBlocks = 2048;           // workgroups of the H_nd pass

void set_error(const std::string& msg);

#define EDX_HIP(call)                                                        \
  do {                                                                       \
    hipError_t e_ = (call);                                                  \
    if (e_ != hipSuccess) {                                                  \
      ::edx::set_error(std::string(#call) + ": " + hipGetErrorString(e_));   \
      return EDX_E_DEVICE;                                                   \
    }                                                                        \
  } while (0)

#define EDX_TRY(expr)               \
  do {                              \
    edx_status s_ = (expr);         \
    if (s_ != EDX_OK) return s_;    \
  } while (0)

// Device memory source of a sector's tables: hipMalloc/hipFree by default; the
// request server hands out pieces of a request's reserved block instead, so
// that no hipFree (which waits for the device) runs while other requests'
// kernels are in flight.
struct Allocator {
  void* (*alloc)(void* ctx, size_t bytes) = nullptr;   // nullptr on failure
  void (*release)(void* ctx, void* p) = nullptr;
  void* ctx = nullptr;
};

// Host copy of the model (arrays owned).
struct Model {
  int norb = 0, nbath = 0, ns = 0;
  std::vector<double> eps_imp, eps_bath, vhyb;
  double U = 0, Ust = 0, Jh = 0, xmu = 0;
  double Jx = 0, Jp = 0;   // spin exchange, pair hopping (eq. Ham1)
  int nph = 0;             // phonon cutoff N_ph (0: no phonons)
  double w0 = 0;           // phonon frequency
  double g[kMaxNorb] = {0, 0, 0};   // electron-phonon couplings g_a
};

// Tables of one spin species of a sector, device resident.
struct SpinTables {
  int n = 0;              // electrons of this spin
  bool orb = false;       // orbital-resolved: counts[a] electrons in orbital a
  int counts[kMaxNorb] = {0, 0, 0};
  int64_t D = 0;          // number of strings
  int width = 0;          // max hops in any row
  int wpad = 8;           // row stride of the hop table: 8, 16 or 24 entries
  int64_t nnz = 0;        // non-padding hop entries
  uint32_t* map = nullptr;    // [D] ascending strings
  int32_t* rank = nullptr;    // [2^Ns] index of a string, -1 if other popcount
  uint32_t* hop = nullptr;    // [D * wpad] packed, row-major: hop[i*wpad + k]
  double* e64 = nullptr;      // [D] diagonal energy
  float* e32 = nullptr;       // [D] same, rounded
  uint8_t* pat = nullptr;     // [D] impurity pattern
};

// Launch plan of edx_hv (see edx_hv_plan).
struct HvPlan {
  int mode = 0;      // 0 small (whole sector in LDS), 1 two-pass, 2 fused column
  int col_cols = 1;  // columns per block in the column pass
  int col_threads = 512;
  int row_rows = 64; // rows per slab in the row pass
  int row_cols = 16; // columns per block in the row pass
  int col_order = 0; // fused pass: 0 natural, 1 XCD-contiguous, 2 + pattern-sorted
  int col_blocks = 0;  // blocks of the last pass (partial count)
};

}  // namespace edx

struct edx_sector {
  edx::Model model;
  edx::Allocator alloc;      // where the device tables came from
  int nup = 0, ndw = 0;
  int64_t dup = 0, ddw = 0, dim = 0;
  bool nd = false;           // spin exchange / pair hopping present (norb >= 2)
  int64_t ld = 0;            // column stride of the library's Krylov vectors
  int64_t vlen = 0;          // ld * ddw * dph elements per Krylov vector
  int dph = 1;               // phonon states N_ph + 1 (1: no phonons); slowest index
  int device = 0;
  edx::SpinTables up, dw;
  // Signed amplitudes indexed by (hop entry >> 24); identical for both spins.
  double* amp64 = nullptr;   // [256] device
  float* amp32 = nullptr;    // [256] device
  // W[p_up * 8 + p_dw]: density-density energy of two impurity patterns.
  double* zeros = nullptr;   // max(D_up, D_dw) + 64 zero doubles (block passes)
  // hop rows in 3 * wpad bytes for the fused pass (spin up) and the column
  // pass on the transposed vector (spin down), built when D < 2^16: wpad
  // 16-bit columns, then wpad 8-bit amplitude indices
  uint8_t* hrow = nullptr;
  uint8_t* hrow_dw = nullptr;
  double* w64 = nullptr;     // [64] device
  float* w32 = nullptr;      // [64] device
  int32_t* binom = nullptr;  // [25*25] device binomial table
  double amp_host[edx::kAmpTable];
  // launch plans of edx_hv per vtype (set by the autotuner or the caller)
  bool plan_set[2] = {false, false};
  edx::HvPlan plan[2];
  // spin-down strings (columns of V) stably sorted by impurity pattern: the
  // column order of the fused pass with col_order 2
  int32_t* corder = nullptr;   // [ddw] device
  // spin exchange / pair hopping terms by impurity-pattern pair (pu, pd):
  // entries nd_off[pu * P + pd] .. nd_off[pu * P + pd + 1] (P = 2^norb) give the
  // source offsets (rows du, columns dd) and signed amplitudes
  int32_t* nd_off = nullptr;   // [P*P + 1] device
  int32_t* nd_du = nullptr;    // [terms]
  int32_t* nd_dd = nullptr;
  double* nd_amp64 = nullptr;
  float* nd_amp32 = nullptr;
  int nd_nt = 0;               // number of terms in the table
  // with phonons: per phonon slice p a term table of the same form for the
  // fused pass (the H_nd terms plus (0, -+D_dw, G(pu, pd) sqrt(p or p+1)):
  // the neighbouring slices are D_dw columns away) and W + w0 p
  int32_t* ph_off = nullptr;   // [dph][P*P + 1], relative to the slice's first term
  int32_t* ph_du = nullptr;
  int32_t* ph_dd = nullptr;
  double* ph_amp64 = nullptr;
  float* ph_amp32 = nullptr;
  std::vector<int> ph_start;   // host: first term of slice p, [dph + 1]
  int ph_nt_max = 0;           // largest per-slice term count
  double* wph64 = nullptr;     // [dph][64]
  float* wph32 = nullptr;
  // lazily built neighbour sectors for the Green's function:
  // [spin][0] = N_s + 1 (particle), [spin][1] = N_s - 1 (hole); for an
  // orbital-resolved sector per orbital: [spin][orb][branch]
  std::mutex nb_mu;
  edx_sector* nb[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
  edx_sector* nb_orb[2][edx::kMaxNorb][2] = {};
  // sectors of the pair operators: [orbital (0 for a total-N sector)][+2 / -2]
  edx_sector* nb_pair[edx::kMaxNorb][2] = {};
  bool orb = false;          // orbital-resolved sector (per-orbital counts)
};

namespace edx {

// ---- tables.hip
// cup/cdw (both or neither): per-orbital electron counts of an orbital-resolved
// sector (nup/ndw are then their sums)
edx_status build_sector_impl(const Model& m, int nup, int ndw, hipStream_t st,
                             edx_sector** out, const Allocator* a = nullptr,
                             const int* cup = nullptr, const int* cdw = nullptr);
// upper bound of the device bytes build_sector_impl takes from an allocator
size_t sector_table_bytes(int ns, int nup, int ndw);
// H_nd term table of a sector with spin exchange / pair hopping
edx_status build_nd_terms(edx_sector* S, const Model& m, const std::vector<int32_t>& binom,
                          hipStream_t st);
void destroy_sector(edx_sector* s);

// ---- hv.hip
HvPlan hv_plan(const edx_sector* s, int vtype);
HvPlan hv_default_plan(const edx_sector* s, int vtype);
edx_status hv_validate(const edx_sector* s, int vtype, HvPlan* p);
// w = H (scale * v), both with column stride ld >= dup; if partial != nullptr
// the last pass writes per-block partial sums of <scale v, w> (FP64) and
// plan.col_blocks of them.
edx_status hv_launch(const edx_sector* s, int vtype, const void* v, void* w, int64_t ld,
                     const double* vscale, double* partial, hipStream_t st,
                     const HvPlan* plan = nullptr);
edx_status hv_autotune(edx_sector* s, int vtype, const void* v, void* w, int64_t ld, int reps,
                       hipStream_t st, HvPlan* best, double* best_us);
int hv_partial_blocks(const edx_sector* s, int vtype);
// per-GPU pieces of the column-distributed product (see edx_hv_block)
edx_status hv_block_launch(const edx_sector* s, int vtype, int part, const void* v, void* w,
                           int64_t ld, int64_t c0, int64_t c1, hipStream_t st);
edx_status k_transpose(int vtype, const void* src, int64_t rows, int64_t cols, int64_t lds,
                       void* dst, int64_t ldd, int add, hipStream_t st);

// ---- krylov.hip
int elem_blocks(int64_t n);
// random start vector in [-1, 1) of the element with logical index r + c*dup
// (the same values for every ld); zero in the padding rows.  With src, the
// dense vector src (dup * ddw elements) is copied into that layout instead.
edx_status k_start_vector(int vtype, void* u, int64_t dup, int64_t ld, int64_t ddw,
                          uint64_t seed, double* partial, hipStream_t st,
                          const void* src = nullptr);
// y[r + c*dup] = scale * x[r + c*ld] (drops the padding rows)
edx_status k_unpad_scale(int vtype, const void* x, int64_t ld, int64_t dup, int64_t ddw,
                         const double* scale, void* y, hipStream_t st);
// reduce `nslots` sets of `nparts` partials (slot-major, stride kMaxPartials)
// into out[0..nslots); op: 0 plain sum, 1 Lanczos alpha, 2 Lanczos beta.
edx_status k_reduce(const double* partial, int nparts, int nslots, double* out,
                    hipStream_t st);
struct LanczosScalars;  // device layout, see krylov.hip
edx_status k_alpha_finish(const double* partial, int nparts, double* alpha_j,
                          hipStream_t st);
edx_status k_beta_finish(const double* partial, int nparts, double* beta_next,
                         double* scale_next, hipStream_t st);
edx_status k_update(int vtype, void* w, const void* vcur, const double* scur,
                    const void* vprev, const double* sprev,
                    const double* alpha, const double* beta, int64_t n,
                    void* psi, const double* ycoef, double* partial,
                    hipStream_t st);
edx_status k_norm2(int vtype, const void* x, int64_t n, double* partial,
                   hipStream_t st);
edx_status k_scale_copy(int vtype, const void* x, const double* scale,
                        void* y, int64_t n, hipStream_t st);
edx_status k_dot2(int vtype, const void* w, const void* a, const double* sa,
                  const void* b, const double* sb, int64_t n, double* partial,
                  hipStream_t st);
edx_status k_axpy2(int vtype, void* w, const void* a, const double* ca,
                   const double* sa, const void* b, const double* cb,
                   const double* sb, int64_t n, double* partial,
                   hipStream_t st);
edx_status k_multi_dot(int vtype, const void* basis, int64_t ld, int m,
                       const void* w, int64_t n, double* partial,
                       hipStream_t st);
edx_status k_multi_axpy(int vtype, void* w, const void* basis, int64_t ld,
                        int m, const double* coef, int64_t n, double* partial,
                        hipStream_t st);
int multi_blocks(int64_t n);
// thick restart: basis_c <- sum_{j<m} C[j*l + c] basis_j for c < l, in place
constexpr int kMaxKeep = 32;
edx_status k_basis_rotate(int vtype, void* basis, int64_t ld, int m, int l, const double* C,
                          int64_t n, hipStream_t st);

// ---- green.hip
// coefficients of a diagonal operator O = sum_a (up[a] n_{a up} + dw[a] n_{a dw})
struct DiagCoef {
  double up[kMaxNorb];
  double dw[kMaxNorb];
};
// phi = (O - *mean) psi (mean != nullptr, partial: |phi|^2) or partial sums of
// <psi|O|psi> (mean == nullptr); nblocks <= kMaxPartials workgroups of 256
edx_status k_diag_apply(const edx_sector* s, int vtype, const void* psi, void* phi,
                        const DiagCoef& c, const double* mean, double* partial, int nblocks,
                        hipStream_t st);
edx_status k_apply_op(const edx_sector* src, const edx_sector* dst, int vtype,
                      const void* psi, void* phi, int orb, int spin, int create,
                      hipStream_t st);
edx_status k_green_cf(const double* ap, const double* bp, int np, double wp,
                      const double* ah, const double* bh, int nh, double wh,
                      double e0, double beta, int lmats, double* g,
                      hipStream_t st, int bosonic = 0);
// phi = (O_exc - *mean) psi (or partials of <psi|O_exc|psi> when mean == nullptr),
// O_exc = sum_sigma (c+_a c_b + c+_b c_a), impurity levels a < b, same sector
edx_status k_exc_apply(const edx_sector* s, int vtype, const void* psi, void* phi, int a,
                       int b, const double* mean, double* partial, int nblocks, hipStream_t st);
// phi (sector dst) = c+_{a up} c+_{a dw} psi (create) or c_{a dw} c_{a up} psi
edx_status k_pair_apply(const edx_sector* src, const edx_sector* dst, int vtype, const void* psi,
                        void* phi, int a, int create, hipStream_t st);

// ---- batch.hip
edx_status batch_run(const edx_sector* const* secs, int n, const edx_lanczos_opts* o,
                     const int* ccols, const int* rcols, int L, int64_t wide_min, int multi_k,
                     void* ws, size_t ws_bytes, edx_batch_result* res, hipStream_t st,
                     double* elapsed_ms);
size_t batch_workspace_bytes(const edx_sector* const* secs, int n, int vtype, int L,
                             int64_t wide_min);
edx_status batch_autotune(const edx_sector* const* secs, int n, const edx_lanczos_opts* o,
                          void* ws, size_t ws_bytes, int* ccols, int* rcols, int* lane_wgs,
                          int64_t* wide_min, hipStream_t st);

// ---- lanczos.hip
size_t lanczos_workspace_bytes(const edx_sector* s, int vtype, int niter, int reorth);
edx_status lanczos_ground_state_impl(const edx_sector* s, const edx_lanczos_opts* o, void* ws,
                                     size_t ws_bytes, double* e0, void* psi0,
                                     edx_lanczos_report* rep, hipStream_t st);
// ---- multi.hip: K bath sets of one sector shape at once (interleaved vectors)
bool multi_supported(const edx_sector* s, int K, int vtype);
bool multi_same_shape(const edx_sector* a, const edx_sector* b);
size_t multi_workspace_bytes(const edx_sector* s, int K, int vtype, int niter);
edx_status multi_ground_states(const edx_sector* const* secs, int K, const edx_lanczos_opts* o,
                               void* ws, size_t ws_bytes, edx_batch_result* res, hipStream_t st);
size_t multi_hv_workspace_bytes(const edx_sector* s, int K, int vtype);
edx_status multi_hv(const edx_sector* const* secs, int K, int vtype, const void* v, void* w,
                    void* ws, size_t ws_bytes, hipStream_t st);

// ---- noalloc.hip: the same ground state with the workspace in a fixed
// per-device scratch array (no device allocation)
edx_status lanczos_ground_state_static(const edx_sector* s, const edx_lanczos_opts* o,
                                       double* e0, void* psi0, edx_lanczos_report* rep,
                                       hipStream_t st);
size_t lowest_workspace_bytes(const edx_sector* s, int vtype, int niter, int k);
edx_status lowest_states_impl(const edx_sector* s, int k, const edx_lanczos_opts* o, int verify,
                              void* ws, size_t ws_bytes, double* e, void* psi,
                              edx_lowest_report* rep, hipStream_t st);
size_t green_workspace_bytes(const edx_sector* s, int vtype, int ngf);
edx_status green_cf_impl(const edx_sector* gs, const void* psi0, double e0, int orb, int spin,
                         const edx_gf_opts* o, void* ws, size_t ws_bytes, double* g_host,
                         edx_gf_report* rep, hipStream_t st);
size_t chi_workspace_bytes(const edx_sector* s, int vtype, int ngf);
// op 0: diagonal density operator c; op 1: excitonic operator of levels a < b
edx_status chi_impl(const edx_sector* s, const void* psi0, double e0, const DiagCoef& c,
                    const edx_gf_opts* o, void* ws, size_t ws_bytes, double* chi_host,
                    edx_chi_report* rep, hipStream_t st, int op = 0, int a = 0, int b = 1);
size_t pair_workspace_bytes(const edx_sector* s, int vtype, int ngf);
edx_status pair_impl(const edx_sector* gs, const void* psi0, double e0, int a,
                     const edx_gf_opts* o, void* ws, size_t ws_bytes, double* chi_host,
                     edx_gf_report* rep, hipStream_t st);
// ---- lanczos.cpp (host)
double tridiag_lowest(const double* a, const double* b, int m, int k);
void tridiag_vector(const double* a, const double* b, int m, double lam,
                    double* y);
bool tridiag_spectrum(const double* a, const double* b, int m, double* theta, double* w);

inline int wpad_of(int width) { return width <= 8 ? 8 : (width <= 16 ? 16 : 24); }
// Column stride of the library's Krylov vectors for a sector with dup rows:
// rounded up to 32 elements (every column starts on a 128-byte line), dense
// for short columns where the padding would cost more than it saves.
inline int64_t vec_ld(int64_t dup) { return dup < 256 ? dup : (dup + 31) / 32 * 32; }
inline size_t vbytes(int vtype) { return vtype == EDX_F32 ? 4 : 8; }
inline size_t align_up(size_t x, size_t a = 256) { return (x + a - 1) / a * a; }

}  // namespace edx
