/*
 * edx.h -- C ABI of the MI355X exact-diagonalisation hot path.
 *
 * The library computes, for an Anderson impurity model with a normal bath and a
 * density-density interaction (eq. Ham1), in one sector of fixed (N_up, N_dw)
 * (Sec. 2.2), the storage-free product w = H v with the decomposition
 * H = H_d + H_up (x) 1 + 1 (x) H_dw (eq. Hdecomp, eq. Hbuild), the Lanczos ground
 * state (Sec. 6 "Diagonalization") and the impurity Green's function by the
 * Krylov continued fraction (Sec. 6 "Dynamical correlation functions").
 *
 * Conventions (every index is 0-based; the paper's are 1-based):
 *   - level k of spin s: impurity orbital a at level a, bath level (a, nu) at
 *     level norb + a*nbath + nu.  Spin strings are Ns-bit integers, bit k =
 *     occupation of level k.  All spin-up modes precede all spin-down modes in
 *     the fermionic order (Sec. 2.3).
 *   - the strings of one spin in a sector are the Ns-bit integers with the
 *     right popcount in ascending order (the build_sector listing of Sec. 6
 *     "Sector construction"); map_s[i] is the i-th one.
 *   - sector index i = i_up + i_dw * D_up: a vector is the D_up x D_dw
 *     column-major matrix of eq. Vmatrix, spin-up fastest, dense, no padding.
 *   - the interaction is plain U n_up n_dw (no Hartree constant); xmu shifts
 *     the impurity levels only.
 *
 * Memory and ownership: model arrays are host memory, copied at build time.
 * Vectors, workspaces and psi0 are device memory owned by the caller; hip
 * streams are the caller's (NULL = default stream).  The library owns the
 * opaque sector handle and its device tables.  edx_hv allocates nothing.
 *
 * Errors: every call returns an edx_status; edx_last_error() gives a
 * thread-local message for the last failing call on this thread.  Nothing
 * crosses the ABI as an exception.  One sector handle may be used from
 * several streams at once for edx_hv (it is read-only after build); the
 * Lanczos and Green calls use only the workspace they are given.
 */
#ifndef EDX_H
#define EDX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  EDX_OK = 0,
  EDX_E_INVALID = 1,     /* bad argument, empty or impossible sector        */
  EDX_E_NOMEM = 2,       /* workspace too small / device allocation failed  */
  EDX_E_DEVICE = 3,      /* a HIP runtime call failed                       */
  EDX_E_NOCONV = 4,      /* Lanczos did not meet its stop rule in niter     */
  EDX_E_DEGENERATE = 5,  /* ground state gap below 1e-9 (flag, e0 is valid) */
  EDX_E_UNSUPPORTED = 6, /* outside the implemented model space            */
  EDX_PENDING = 7        /* edx_server_poll without wait: not finished yet  */
} edx_status;

/* storage type of v, w, Krylov vectors and psi0; scalars are always FP64 */
typedef enum { EDX_F64 = 0, EDX_F32 = 1 } edx_vtype;

/* Normal-bath impurity model of eq. Ham1: one-body levels, hybridisation,
 * the density-density interaction, and the spin-exchange and pair-hopping
 * terms  - Jx sum_{a!=b} d+_{a up} d_{a dw} d+_{b dw} d_{b up}
 *        + Jp sum_{a!=b} d+_{a up} d+_{a dw} d_{b dw} d_{b up}
 * on the impurity orbitals (Jx = Jp = 0: density-density only).
 * Ns = norb*(nbath+1) must be <= 24, norb <= 3. */
typedef struct {
  int32_t norb;
  int32_t nbath;
  const double* eps_imp;   /* [norb]                       host */
  const double* eps_bath;  /* [norb*nbath], orbital-major host */
  const double* vhyb;      /* [norb*nbath], orbital-major host */
  double U;                /* intra-orbital n_up n_dw                    */
  double Ust;              /* U': inter-orbital opposite spin            */
  double Jh;               /* J: same-spin inter-orbital gets U' - J     */
  double xmu;              /* chemical potential on the impurity levels  */
  double Jx;               /* spin exchange J_X                          */
  double Jp;               /* pair hopping J_P                           */
  /* Holstein phonon (Sec. "Electron-phonon coupling"):
   *   H += w0 b+b + sum_{a sigma} g_a n_{a sigma} (b + b+),
   * one local mode truncated at nph quanta (0 = no phonons, at most 63).
   * A sector is then the electronic sector times D_ph = nph + 1 phonon
   * states, index i = i_up + D_up (i_dw + D_dw p) (eq. HephBuild), and every
   * vector of it is D_ph electronic vectors one after another. */
  int32_t nph;
  int32_t pad_;
  double w0;               /* phonon frequency                           */
  const double* g;         /* [norb] couplings g_a (NULL when nph = 0)   */
} edx_model;

typedef struct edx_sector edx_sector;
typedef struct edx_server edx_server;

/* Build the tables of sector (nup, ndw) on the current device (Sec. 6 "Sector
 * construction", eq. nud_dimension): per spin the ascending string map, its
 * inverse over all 2^Ns integers, the hopping lists with fermionic signs
 * (Sec. 2.3) and the diagonal tables (eq. Hbuild).  Runs kernels on `stream`
 * and returns after they finish.  nup/ndw outside [0, Ns] -> EDX_E_INVALID. */
edx_status edx_build_sector(const edx_model* model, int32_t nup, int32_t ndw,
                            void* stream, edx_sector** out);

/* Orbital-resolved sector (Sec. 2.2, eqs. Fock_decomp and Irelation with
 * N_ud = N_alpha; Sec. 2.3, the split of H_sigma into per-orbital terms):
 * nup[a], ndw[a] (host, [norb]) electrons of each spin among orbital a's
 * N_bit = nbath + 1 levels (its impurity level, then its bath levels).  Per
 * spin, orbital a's local string has its ascending (colex) position r_a and
 * the string index is r_1 + D_1 (r_2 + D_2 r_3), D_a = C(nbath+1, counts[a]).
 * The sector is used like one from edx_build_sector (the same H.v, Lanczos and
 * Green's function entry points); its Green's function neighbours change
 * only orbital orb's count.  The conservation needs H_nd = 0: Jx or Jp != 0
 * -> EDX_E_UNSUPPORTED; a count outside [0, nbath+1] or a NULL array ->
 * EDX_E_INVALID. */
edx_status edx_build_sector_orbital(const edx_model* model, const int32_t* nup,
                                    const int32_t* ndw, void* stream, edx_sector** out);

void edx_sector_destroy(edx_sector* s);

/* D_up, D_dw and D = D_up * D_dw of a sector (eq. nud_dimension). */
edx_status edx_sector_dims(const edx_sector* s, int64_t* dup, int64_t* ddw,
                           int64_t* dim);

/* Column stride (in elements) that the library's own Krylov vectors use for
 * this sector: D_up rounded up to a multiple of 32 (every column of V, eq.
 * Vmatrix, then starts on a 128-byte line), or D_up itself for D_up < 256.
 * Passing it as `ld` to edx_hv gives the fastest product. */
edx_status edx_sector_ld(const edx_sector* s, int64_t* ld);

/* Number of hopping entries of one spin (0 = up, 1 = down) and the largest
 * number in any row. */
edx_status edx_sector_hop_nnz(const edx_sector* s, int32_t spin, int64_t* nnz,
                              int32_t* max_row);

/* Host copies of one spin's tables, for tests.  Any pointer may be NULL.
 *   map[D_s]           ascending strings
 *   hop_off[D_s + 1]   CSR row offsets; row i lists j with <i|H_s|j> != 0
 *   hop_col[nnz]       column j, ascending within a row
 *   hop_sign[nnz]      +1 / -1: (-1)^(occupied levels strictly between the
 *                      two levels of the hop), Sec. 2.3
 *   hop_amp[nnz]       sign * V of the hop
 *   diag_e[D_s]        one-body energy + same-spin inter-orbital term
 *   diag_p[D_s]        impurity occupation pattern (bits 0..norb-1) */
edx_status edx_sector_get_tables(const edx_sector* s, int32_t spin,
                                 uint32_t* map, int64_t* hop_off,
                                 int32_t* hop_col, int8_t* hop_sign,
                                 double* hop_amp, double* diag_e,
                                 uint8_t* diag_p);

/* Host copy of one spin's inverse map over all 2^Ns integers (Sec. 6
 * "Sector construction": the position of a string in the ascending listing,
 * found there by binary search; here tabulated from the colex rank, or for an
 * orbital-resolved sector from the mixed-radix index of Sec. 2.2):
 * rank[s] = i when map[i] == s, -1 for strings outside the sector's spin
 * species.  rank must hold 2^Ns int32 values. */
edx_status edx_sector_get_rank(const edx_sector* s, int32_t spin, int32_t* rank);

/* w = H v for the sector (Sec. 3 MVP, eq. Hbuild; storage-free, Sec. 2.4).
 * v and w are device arrays of `vtype` holding the D_up x D_dw matrix V of
 * eq. Vmatrix column by column with column stride `ld` (0 = dense, D_up;
 * otherwise ld >= D_up, ld * D_dw elements per array).  Rows D_up..ld-1 of v
 * are not read; those of w are written as zero.  v and w must not overlap and
 * are accessed on `stream`.  Enqueues kernels and returns; allocates nothing.
 * ld in (0, D_up) -> EDX_E_INVALID. */
edx_status edx_hv(const edx_sector* s, edx_vtype vtype, const void* v, void* w,
                  int64_t ld, void* stream);

/* Launch plan of edx_hv (tile shapes; the result is the same for every plan up
 * to rounding order).  mode 0: whole sector in LDS, one block; mode 1: two
 * passes (spin-down rows, then spin-up columns + diagonal); mode 2: one pass
 * over columns that also gathers the spin-down neighbours from global memory.
 * col_cols: columns per block (1..4) of the column pass; col_threads: 256, 512
 * or 1024; row_rows: rows per slab (16, 32, 64, or 128 = two rows per lane,
 * even D_up only); row_cols: columns per block of the row pass (>= 1);
 * col_order (mode 2): which columns a workgroup takes -- 0 consecutive groups
 * in workgroup order, 1 the groups running at once on one XCD are
 * consecutive, 2 as 1 over the columns sorted by impurity occupation (so
 * that concurrently processed columns share more spin-down neighbours), 3 and
 * 4 as 1 and 2 inside windows of about one group per CU (3) or two (4) that
 * all XCDs walk together (their neighbour columns then also meet in the
 * MALL). */
typedef struct {
  int32_t mode, col_cols, col_threads, row_rows, row_cols, col_order;
} edx_hv_plan;

/* Current plan of a sector for one vtype (the built-in heuristic until set). */
edx_status edx_hv_get_plan(const edx_sector* s, edx_vtype vtype, edx_hv_plan* plan);
/* Replace the plan (validated; EDX_E_INVALID / EDX_E_UNSUPPORTED if it cannot
 * run on this sector).  Not thread-safe against concurrent edx_hv calls. */
edx_status edx_hv_set_plan(edx_sector* s, edx_vtype vtype, const edx_hv_plan* plan);
/* Project autotuner: times every candidate plan with `reps` launches on the
 * caller's v, w (device, column stride ld as for edx_hv) and keeps the
 * fastest in the sector.  The Lanczos and Green calls use that plan with the
 * stride of edx_sector_ld, so tune with that stride. */
edx_status edx_autotune_hv(edx_sector* s, edx_vtype vtype, const void* v, void* w,
                           int64_t ld, int32_t reps, void* stream, edx_hv_plan* best,
                           double* best_us);

typedef struct {
  int32_t niter;        /* max steps, default 512 (lanc_niter)              */
  int32_t vtype;        /* edx_vtype of the Krylov vectors and psi0         */
  int32_t reorth;       /* 0 none (plain, as the paper), 1 local, 2 full,
                           3 none with the basis kept: psi0 from the stored
                           vectors instead of a replay of the recurrence
                           (niter + 1 vectors of workspace)                  */
  int32_t check_every;  /* host stop-rule check period in steps (>= 1)      */
  double tol;           /* stop if |E_j - E_{j-1}| <= tol * max(1, |E_j|)   */
  double rtol;          /* and (if > 0) beta_{j+1}|y_j| <= rtol * max(1,|E|) */
                        /* with FP32 vectors both thresholds are floored at
                           2 * 2^-23 * |T| (the energy resolution of FP32)    */
  uint64_t seed;        /* SplitMix64 seed of the start vector              */
  int32_t degen_check;  /* ground-state degeneracy check (default 1): after
                           psi0 is formed, a second Lanczos run kept
                           orthogonal to psi0 finds the lowest level of the
                           complement; a level within gs_threshold =
                           1e-9 max(1, |E0|) of E0 (FP32 vectors: at least
                           2 * 2^-23 |T|) makes the ground level degenerate.
                           Runs only when psi0 is requested.               */
  int32_t pad_;
  const void* start;    /* nullable: a dense device vector (D elements of
                           vtype, any nonzero norm) used as the start vector
                           instead of the SplitMix64 one -- e.g. an FP32
                           ground vector, cast to FP64, to refine it in FP64
                           with a few steps.  Ground state only; must not
                           alias psi0.  Zero or non-finite: EDX_E_INVALID.  */
} edx_lanczos_opts;

typedef struct {
  int32_t iters;        /* Lanczos steps taken                              */
  int32_t converged;    /* 1 if the stop rule was met                       */
  int32_t breakdown;    /* 1 if beta fell below 1e-12 * |T|                 */
  int32_t degenerate;   /* 1 if the ground level is degenerate (see
                           degen_check; without the check: a second Ritz
                           value of the run within 1e-9 of E0)             */
  double e0, e1;        /* E0 and the next level: with the check the lowest
                           level orthogonal to psi0 (a second copy of E0
                           when degenerate), else the second Ritz value    */
  double beta_last;     /* last beta                                        */
  double resid;         /* beta_{m} |y_{m-1}|                               */
} edx_lanczos_report;

void edx_lanczos_default_opts(edx_lanczos_opts* o);

#define EDX_WS_LANCZOS 0
#define EDX_WS_GREEN 1
#define EDX_WS_LANCZOS_BASIS 2

/* Device workspace bytes for edx_lanczos_ground_state (what = EDX_WS_LANCZOS,
 * n = niter; what = EDX_WS_LANCZOS_BASIS = 2 for reorth 2 or 3), edx_green_cf (what = EDX_WS_GREEN, n = ngf), edx_chi and
 * edx_chi_exciton (what = EDX_WS_CHI = 3, n = ngf) or edx_chi_pair
 * (what = EDX_WS_PAIR = 4, n = ngf). */
size_t edx_workspace_bytes(const edx_sector* s, int32_t what, int32_t vtype,
                           int32_t n);

/* Lowest eigenpair of the sector by Lanczos (Sec. 6 "Diagonalization"):
 * alpha_j = <v_j, H v_j>, w = H v_j - alpha_j v_j - beta_j v_{j-1},
 * beta_{j+1} = |w|, v_{j+1} = w / beta_{j+1}; scalars and dots in FP64.
 * psi0 (nullable, D elements of opts->vtype) receives the normalised ground
 * vector from a second replay of the same recurrence.  A run from one start
 * vector sees one vector of a degenerate level; with psi0 requested and
 * opts->degen_check set, a further run deflated against psi0 tests the
 * ground level against the degeneracy threshold gs_threshold (Appendix A,
 * 1e-9), and rep->e1 receives its lowest level.  Returns EDX_OK,
 * EDX_E_NOCONV (e0 is the best estimate) or EDX_E_DEGENERATE (e0 and psi0
 * are valid; psi0 is one vector of the degenerate level, and quantities that
 * must average over the level, such as G, go through the eigenstate list,
 * edx_espace_*). */
edx_status edx_lanczos_ground_state(const edx_sector* s,
                                    const edx_lanczos_opts* opts, void* ws,
                                    size_t ws_bytes, double* e0, void* psi0,
                                    edx_lanczos_report* rep, void* stream);

/* The same ground state for callers that cannot allocate device memory
 * (code under stream capture, tight serving loops, harnesses that forbid
 * hipMalloc): identical arguments, checks and results to
 * edx_lanczos_ground_state, but the workspace is a fixed 256 MiB array per
 * GPU inside the library (held from the first call on that GPU until the
 * process ends) instead of a caller buffer, and the call itself allocates
 * nothing.  The sector's device must be the current device.  A sector whose
 * workspace (edx_workspace_bytes, what = EDX_WS_LANCZOS, or
 * EDX_WS_LANCZOS_BASIS for reorth 2 and 3) exceeds 256 MiB -> EDX_E_NOMEM.
 * Every call on one GPU uses the same array: calls that overlap on one GPU
 * (from several host threads or streams) race and must be serialised by the
 * caller. */
edx_status edx_lanczos_ground_state_static(const edx_sector* s,
                                           const edx_lanczos_opts* opts, double* e0,
                                           void* psi0, edx_lanczos_report* rep,
                                           void* stream);

/* ---- several bath sets of one sector shape at once (the paper's
 * independent impurity problems, Sec. 6 "Main", solved together) ----
 * k (1, 2, 4 or 8) sectors with the same Ns, Norb, N_up and N_dw (the same
 * strings, hop columns and signs: the tables of secs[0] serve all) and their
 * own baths and interaction.  v and w hold the k vectors interleaved element
 * by element: element (i, j) of set b (row i of column j of eq. Vmatrix) at
 * (i + j ld) k + b, ld = edx_sector_ld of the sectors, ld * D_dw * k elements
 * each (padding rows of v not read, of w written as zero).  w_b = H_b v_b for
 * every set, with each set's H v summed exactly as edx_hv's fused pass with one
 * column per workgroup; one spin-down gather serves all k sets.  ws: device
 * workspace of edx_hv_multi_workspace_bytes (the per-set tables and partial
 * sums; each call copies the k sets' tables into it on the stream first).
 * Faster per vector than k separate edx_hv calls only on small sectors
 * (measured: half-filled Ns=12, 1.9x in FP32); from Ns=14 on the single-set
 * pass is faster, because interleaving does not reduce the bytes that cross
 * L2 per vector.  Total-N sectors without spin exchange, pair hopping or phonons,
 * hop rows of 8 or 16 entries, D_up < 2^16, a column of the k sets within LDS
 * and 32-bit byte offsets; otherwise EDX_E_UNSUPPORTED.  Sectors of different
 * shapes -> EDX_E_INVALID. */
size_t edx_hv_multi_workspace_bytes(const edx_sector* const* secs, int32_t k, int32_t vtype);
edx_status edx_hv_multi(const edx_sector* const* secs, int32_t k, edx_vtype vtype,
                        const void* v, void* w, void* ws, size_t ws_bytes, void* stream);

/* ---- the per-GPU pieces of the column-distributed product (Sec. 3.2:
 * columns of V split over processes, two transposes per product), callable on
 * one GPU so that a sharded product can be composed and its per-GPU work
 * measured at the real block shapes.
 * part 0: w[:, c0:c1] = H_d o V[:, c0:c1] + H_up V[:, c0:c1] for the column
 *         block [c0, c1) of V (D_up x D_dw, column stride ld >= D_up);
 * part 1: w[:, c0:c1] = H_dw VT[:, c0:c1] for the column block [c0, c1) of the
 *         transposed vector VT (D_dw x D_up, column stride ld >= D_dw), i.e. the
 *         spin-down hops made local by the transpose (no diagonal).
 * Output columns are overwritten, their padding rows written as zero; other
 * columns are untouched.  With phonons, apply per phonon slice.
 * EDX_E_INVALID for a bad part, range or ld. */
edx_status edx_hv_block(const edx_sector* s, edx_vtype vtype, int32_t part, const void* v,
                        void* w, int64_t ld, int64_t c0, int64_t c1, void* stream);

/* dst (cols x rows, column stride ldd >= cols) = src^T, or dst += src^T when
 * add = 1; src is rows x cols with column stride lds >= rows (device, vtype
 * elements).  The local part of the all-to-all transpose of Sec. 3.2. */
edx_status edx_transpose(edx_vtype vtype, const void* src, int64_t rows, int64_t cols,
                         int64_t lds, void* dst, int64_t ldd, int32_t add, void* stream);

/* ---- several low-lying states (Sec. 6 "Eigenspace class": lanc_nstates_*)
 * The k lowest eigenpairs of one sector by Lanczos with full
 * re-orthogonalisation and locking: each run starts from a random vector
 * (SplitMix64, seed + run) orthogonal to the states locked so far, keeps
 * every new Krylov vector orthogonal to them and to the run's own basis
 * (classical Gram-Schmidt twice), and locks the lowest Ritz pairs whose
 * residual beta_m |y_{m-1}| <= rtol max(1, |theta|) (tol when rtol = 0; FP32
 * floor as for the ground state).  A run aims at min(k - locked, niter/4)
 * states; when its basis reaches niter first it is thick-restarted in place
 * (the lowest l <= 32 Ritz vectors kept, the arrow matrix they give brought
 * back to tridiagonal form, at most 64 restarts a run), so niter bounds the
 * basis memory, not the number of steps.  A run from one start vector sees one
 * vector per degenerate eigenspace; the locking finds the other copies in
 * later runs, and with verify = 1 a last run checks that the lowest state
 * orthogonal to all k locked ones lies at or above the k-th energy (a lower
 * one replaces the highest and the check repeats).  k is clipped to D.
 * e (host, [k]) ascending; psi (device, nullable) receives the k normalised
 * vectors, dense, one after another (k * D elements of opts->vtype).
 * opts->reorth is ignored.  EDX_OK, or EDX_E_NOCONV with the states found. */
typedef struct {
  int32_t nfound;       /* states returned (k clipped to D)                 */
  int32_t runs;         /* Lanczos runs (restarts and the check included)   */
  int32_t iters;        /* Lanczos steps over all runs                      */
  int32_t verified;     /* 1 if the check run passed (or verify = 0)        */
  double resid_max;     /* largest residual estimate of a locked pair       */
} edx_lowest_report;

#define EDX_MAX_STATES 64

size_t edx_lowest_workspace_bytes(const edx_sector* s, int32_t vtype, int32_t niter,
                                  int32_t k);

edx_status edx_lanczos_lowest(const edx_sector* s, int32_t k,
                              const edx_lanczos_opts* opts, int32_t verify,
                              void* ws, size_t ws_bytes, double* e, void* psi,
                              edx_lowest_report* rep, void* stream);

typedef struct {
  int32_t ngf;     /* Krylov depth per branch (lanc_ngfiter), default 200 */
  int32_t lmats;   /* number of Matsubara frequencies                   */
  int32_t vtype;   /* storage of the Krylov vectors (psi0 has this type) */
  int32_t pad_;
  double beta;     /* inverse temperature of w_n = (2n+1) pi / beta      */
} edx_gf_opts;

typedef struct {
  double wp, wh;       /* |c+ psi0|^2 and |c psi0|^2                      */
  int32_t np, nh;      /* recurrence lengths of the two branches          */
  double* alpha_p;     /* optional host outputs [ngf] (may be NULL)       */
  double* beta_p;      /* beta_p[k] couples steps k and k+1, [ngf]        */
  double* alpha_h;
  double* beta_h;
} edx_gf_report;

/* Impurity Green's function G(i w_n) of orbital `orb`, spin `spin` at T = 0
 * (eq. KLgf, both fermionic terms +, energies from e0) by the Krylov
 * continued fraction: phi_p = c+ psi0 in (N_s + 1), phi_h = c psi0 in
 * (N_s - 1), ngf plain Lanczos steps per branch,
 *   G = w_p / (z - (a0p - e0) - b1p^2 / (z - (a1p - e0) - ...))
 *     + w_h / (z + (a0h - e0) - b1h^2 / (z + (a1h - e0) - ...)).
 * The (N_s +- 1) sector tables are built on first use and kept with `gs`.
 * g_host receives 2*lmats doubles (re, im interleaved). */
edx_status edx_green_cf(const edx_sector* gs, const void* psi0, double e0,
                        int32_t orb, int32_t spin, const edx_gf_opts* opts,
                        void* ws, size_t ws_bytes, double* g_host,
                        edx_gf_report* rep, void* stream);

/* Poles and weights of a Krylov spectral function (Sec. 6 "Dynamical
 * correlation functions": the eigenvalues theta_m of the Lanczos tridiagonal
 * matrix and the squared first components |a_m|^2 of its eigenvectors).
 * alpha [m] diagonal, beta [m-1] off-diagonal, theta and weight [m] outputs,
 * all host; theta ascending.  Implicit symmetric QR with the Wilkinson shift,
 * O(m^2).  EDX_E_NOCONV if a block does not converge. */
edx_status edx_tridiag_spectrum(const double* alpha, const double* beta, int32_t m,
                                double* theta, double* weight);

/* Density-type susceptibility at T = 0 (eq. KLgf with the bosonic sign, Sec. 6
 * "Dynamical correlation functions"; the paper's spin and charge functions):
 * O = sum_a (cu[a] n_{a up} + cd[a] n_{a dw}) (host arrays [norb]; S_z of
 * orbital a: cu[a] = 1/2, cd[a] = -1/2; charge: 1, 1; a cross-orbital function
 * from O = A + B), diagonal in the occupation basis, so O psi0 stays in the
 * sector of psi0 (dense, D elements of opts->vtype):
 *   C(i nu_n) = sum_m |<m|O|psi0>|^2 [1/(i nu_n - (E_m - E0)) - 1/(i nu_n + (E_m - E0))]
 *             = -sum_m |<m|O|psi0>|^2 2 d_m / (nu_n^2 + d_m^2),  nu_n = 2 n pi / beta,
 * from ngf plain Lanczos steps started at (O - <O>) psi0, with the poles and
 * weights of the tridiagonal matrix.  Poles with |d_m| within gs_threshold =
 * 1e-9 max(1, |E0|) (FP32 vectors: at least 2 * 2^-23 |T|) are dropped: they
 * give 1/z - 1/z = 0 for z != 0 and the T = 0 limit at z = 0 (subtracting <O>
 * psi0 only removes such a pole).  chi_host: 2*lmats doubles (re, im). */
typedef struct {
  double w;          /* |(O - <O>) psi0|^2                                   */
  double mean;       /* <psi0|O|psi0>                                        */
  int32_t n;         /* recurrence length                                     */
  int32_t dropped;   /* poles dropped as zero-energy                          */
} edx_chi_report;

#define EDX_WS_CHI 3

edx_status edx_chi(const edx_sector* s, const void* psi0, double e0, const double* cu,
                   const double* cd, const edx_gf_opts* opts, void* ws, size_t ws_bytes,
                   double* chi_host, edx_chi_report* rep, void* stream);

/* Excitonic susceptibility at T = 0 (the same form as edx_chi): O = sum_sigma
 * (c+_{a sigma} c_{b sigma} + c+_{b sigma} c_{a sigma}) for impurity orbitals
 * a != b, which keeps the sector.  Total-N sectors without phonons (it moves
 * electrons between orbitals, so an orbital-resolved sector is refused with
 * EDX_E_UNSUPPORTED).  Workspace as for edx_chi (EDX_WS_CHI). */
edx_status edx_chi_exciton(const edx_sector* s, const void* psi0, double e0, int32_t a,
                           int32_t b, const edx_gf_opts* opts, void* ws, size_t ws_bytes,
                           double* chi_host, edx_chi_report* rep, void* stream);

/* Pair susceptibility at T = 0 (eq. KLgf with the bosonic sign), O =
 * c_{a dw} c_{a up} of impurity orbital a:
 *   C(i nu_n) = <O 1/(z - (H - E0)) O+> - <O+ 1/(z + (H - E0)) O>,  z = i 2 n pi / beta,
 * from ngf plain Lanczos steps in each of the sectors (N_up + 1, N_dw + 1) and
 * (N_up - 1, N_dw - 1) (orbital-resolved: orbital a's two counts +-1), built on
 * first use and kept with `gs`, and the two continued fractions (the second
 * with a minus sign).  rep: wp = |O+ psi0|^2, wh = |O psi0|^2 and the lengths.
 * Sectors with phonons -> EDX_E_UNSUPPORTED.  Workspace: edx_workspace_bytes
 * with what = EDX_WS_PAIR. */
#define EDX_WS_PAIR 4
edx_status edx_chi_pair(const edx_sector* gs, const void* psi0, double e0, int32_t a,
                        const edx_gf_opts* opts, void* ws, size_t ws_bytes, double* chi_host,
                        edx_gf_report* rep, void* stream);

/* ---- finite temperature: the eigenstate list (Sec. 6 "Eigenspace class"
 * and the thermal form of "Dynamical correlation functions") ----
 * An edx_espace holds the low-lying states of a fixed set of nsec sectors.
 * edx_espace_diag asks sector i for its next_i lowest states
 * (edx_lanczos_lowest, next_i = nstates_sector at first), merges them into one
 * list ordered by energy (ties: sector, then state), E0 = the lowest, and
 * keeps the states with exp(-beta (E - E0)) >= cutoff, at most nstates_total
 * of them (the printed inequality is read as "drop the states whose factor is
 * below the cutoff").  Annealing: a sector whose computed states were all kept
 * asks for nstates_step more at the next call, any other one for the number
 * it kept (at least 1, at most EDX_MAX_STATES); repeated calls settle the
 * distribution.  Kept vectors stay in device memory owned by the espace (one
 * allocation per sector that keeps a state); the sector handles are not owned
 * and must outlive the espace's use of them.  nstates_total = 1 is T = 0. */
typedef struct edx_espace edx_espace;

typedef struct {
  double beta;             /* inverse temperature, k_B = 1 (default 1000)      */
  double cutoff;           /* Boltzmann factor cutoff (default 1e-9)           */
  int32_t nstates_sector;  /* first request per sector (default 2)             */
  int32_t nstates_total;   /* most states in the list (default 1 = T = 0)      */
  int32_t nstates_step;    /* annealing increment (default 2)                  */
  int32_t verify;          /* check run of edx_lanczos_lowest (default 1)      */
} edx_espace_opts;

void edx_espace_default_opts(edx_espace_opts* o);
edx_status edx_espace_create(const edx_espace_opts* o, int32_t nsec, edx_espace** out);
void edx_espace_destroy(edx_espace* E);

/* Workspace for edx_espace_diag with these sectors and the current requests. */
size_t edx_espace_diag_workspace_bytes(const edx_espace* E, edx_sector* const* secs,
                                       int32_t nsec, int32_t vtype, int32_t niter);

/* Diagonalise every sector (secs[i] is slot i; nsec as at creation) and
 * rebuild the list; the previous list and its vectors are released first.
 * opts as for edx_lanczos_lowest; the vectors have opts->vtype.  Stops at the
 * first sector that fails (its status is returned, the list is left empty). */
edx_status edx_espace_diag(edx_espace* E, edx_sector* const* secs, int32_t nsec,
                           const edx_lanczos_opts* opts, void* ws, size_t ws_bytes,
                           void* stream);

/* Kept states, E0 and Z = sum of exp(-beta (E_n - E0)) over them. */
edx_status edx_espace_info(const edx_espace* E, int32_t* nstates, double* e0, double* z);

/* State i of the list (ascending energy): energy, sector slot, weight
 * exp(-beta (E - E0)) / Z and its dense device vector (owned by E). */
edx_status edx_espace_state(const edx_espace* E, int32_t i, double* e, int32_t* sec,
                            double* weight, const void** psi);

/* Per sector: states computed and kept by the last diag, next request. */
edx_status edx_espace_sector(const edx_espace* E, int32_t sec, int32_t* computed,
                             int32_t* kept, int32_t* next);

/* Workspace for edx_espace_green (the largest Green's function workspace over
 * the sectors that keep a state). */
size_t edx_espace_green_workspace_bytes(const edx_espace* E, int32_t ngf);

/* Thermal impurity G(i w_n) = sum_n w_n G_n, w_n = exp(-beta (E_n - E0)) / Z,
 * over the kept states; G_n is edx_green_cf of state n with its own energy
 * E_n as the reference (poles at E_m - E_n).  opts->beta must equal the
 * espace's beta and opts->vtype the vectors' type. */
edx_status edx_espace_green(edx_espace* E, int32_t orb, int32_t spin,
                            const edx_gf_opts* opts, void* ws, size_t ws_bytes,
                            double* g_host, void* stream);

/* Thermal susceptibility sum_n w_n C_n over the kept states, C_n the T = 0
 * form of edx_chi for state n with E_n as reference.  For z != 0 this is the
 * bosonic Lehmann double sum (pairs with equal energies cancel); at nu = 0 the
 * zero-energy terms (beta |<m|O|n>|^2 w_n within a degenerate level) are not
 * included. */
size_t edx_espace_chi_workspace_bytes(const edx_espace* E, int32_t ngf);
edx_status edx_espace_chi(edx_espace* E, const double* cu, const double* cd,
                          const edx_gf_opts* opts, void* ws, size_t ws_bytes,
                          double* chi_host, void* stream);

/* Thermal excitonic and pair susceptibilities, sum_n w_n C_n over the kept
 * states with the T = 0 forms of edx_chi_exciton / edx_chi_pair and E_n as the
 * reference; the same sector restrictions apply to every kept state's sector.
 * Workspaces: edx_espace_chi_workspace_bytes (exciton) and
 * edx_espace_pair_workspace_bytes (pair). */
size_t edx_espace_pair_workspace_bytes(const edx_espace* E, int32_t ngf);
edx_status edx_espace_chi_exciton(edx_espace* E, int32_t a, int32_t b, const edx_gf_opts* opts,
                                  void* ws, size_t ws_bytes, double* chi_host, void* stream);
edx_status edx_espace_chi_pair(edx_espace* E, int32_t a, const edx_gf_opts* opts, void* ws,
                               size_t ws_bytes, double* chi_host, void* stream);

/* ---- batched ground states (many sectors, one persistent launch) ----
 * Every job is an independent sector; the ground energy of each follows the
 * plain recurrence of edx_lanczos_ground_state (psi0 is not formed).  The
 * paper's counterpart is its parallelism over independent impurity problems
 * (Sec. 6 "Main", inequivalent sites).  Jobs with D >= wide_min_dim fill the
 * GPU by themselves: they run first, through the kernels and host stop rule
 * of edx_lanczos_ground_state (tol and rtol) -- jobs of one sector shape up to
 * tiles.multi_k at a time through the multi-set pass (one interleaved product
 * and recurrence per step for the group), the others one by one -- on three
 * streams.  The others
 * share one cooperative launch: lanes of `lane_wgs` workgroups on one XCD
 * each pull jobs (largest first) from a device queue and evaluate the tol
 * stop rule on the device.  A job's status is EDX_OK, EDX_E_NOCONV (e0 is the
 * last estimate) or EDX_E_DEVICE (a lane barrier timed out). */
typedef struct {
  double e0;
  double beta_last;
  int32_t iters;
  int32_t status;
  int32_t breakdown;
  int32_t pad_;
} edx_batch_result;

typedef struct {
  int32_t lane_wgs;       /* workgroups per lane: 8, 16 or 32             */
  int32_t multi_k;        /* whole-GPU jobs of one sector shape (the same
                             Ns, Norb, N_up, N_dw; each its own bath) and
                             at most 2^21 states run up to multi_k at a
                             time (8, 4 or 2; FP64 vectors at most 4)
                             through the multi-set pass of edx_hv_multi,
                             the rest one by one; 0 = 8, 1 = off.  Larger
                             shapes always run one by one: there the
                             single-set pass is faster per vector        */
  const int32_t* ccols;   /* [n] columns per column-pass item (1..4), or NULL (1) */
  const int32_t* rcols;   /* [n] columns per row-pass item, or NULL (32)   */
  int64_t wide_min_dim;   /* jobs with D >= this run first, one at a time
                             through the whole-GPU kernels; 0 = 2,000,000;
                             < 0 = none (every job on a lane)              */
} edx_batch_tiles;

/* Device workspace bytes for n jobs with lanes of lane_wgs workgroups and the
 * given wide threshold (0 = default, < 0 = none). */
size_t edx_batch_workspace_bytes(const edx_sector* const* sectors, int32_t n,
                                 int32_t vtype, int32_t lane_wgs,
                                 int64_t wide_min_dim);

/* Ground energies of n sectors (host array of handles).  opts: niter, vtype,
 * tol, check_every and seed are used, and rtol for the whole-GPU jobs
 * (reorth must be 0).  tiles may be NULL (lane_wgs 32).  results: host array
 * of n.  Blocks until done; elapsed_ms (nullable) receives the device time
 * from the first job's start to the last job's end. */
edx_status edx_batch_ground_state(const edx_sector* const* sectors, int32_t n,
                                  const edx_lanczos_opts* opts,
                                  const edx_batch_tiles* tiles, void* ws,
                                  size_t ws_bytes, edx_batch_result* results,
                                  double* elapsed_ms, void* stream);

/* Project autotuner for the batched launch: per distinct (D_up, D_dw) it
 * times short runs of each (ccols, rcols) candidate on lanes, then each lane
 * size with each whole-GPU threshold (none, 0.25M, 1M, 2M, 4M, 8M); writes
 * ccols[n], rcols[n] (host), *lane_wgs and *wide_min_dim.  Candidates whose
 * workspace exceeds ws_bytes are skipped; ws must hold at least
 * edx_batch_workspace_bytes(..., 32, -1) bytes. */
edx_status edx_batch_autotune(const edx_sector* const* sectors, int32_t n,
                              const edx_lanczos_opts* opts, void* ws,
                              size_t ws_bytes, int32_t* ccols, int32_t* rcols,
                              int32_t* lane_wgs, int64_t* wide_min_dim,
                              void* stream);

/* ---- request server (continuous batching) ----
 * Requests (a model and a sector) arrive at any time; each gets the ground
 * state (edx_lanczos_ground_state, plain recurrence, psi0 by replay) and, if
 * ngf > 0, G(i w_n) of orbital 0, spin up (edx_green_cf).  The server owns one
 * device arena of hbm_budget bytes (allocated at creation; requests allocate
 * nothing else) and max_slots worker threads with their own streams.  A
 * request is admitted when a slot is free and its footprint (tables,
 * workspaces, psi0) fits in the arena; among the pending requests that fit,
 * the smallest footprint goes first (its work is the smallest), one request
 * of 1 GiB or more runs at a time (large requests are bandwidth-bound: one at
 * a time they finish sooner at the same throughput), and a request passed
 * over 8 times goes next, blocking further passing.  Admitted requests
 * overlap on the device; each runs the plain path's kernels, so its result
 * does not depend on what else runs.  Times are seconds of
 * edx_server_clock(). */
typedef struct {
  size_t hbm_budget;          /* arena bytes                                  */
  int32_t max_slots;          /* concurrent requests (1..64)                  */
  int32_t vtype;              /* storage of the Krylov vectors                */
  int32_t ngf;                /* Green's-function depth; 0 = ground state only */
  int32_t lmats;              /* Matsubara frequencies                        */
  double beta;                /* inverse temperature of the Matsubara grid    */
  edx_lanczos_opts lanczos;   /* niter, tol, rtol, check_every, seed          */
} edx_server_opts;

typedef struct {
  int64_t ticket;
  int32_t status;             /* of the request's ground state / Green call   */
  int32_t iters;
  double e0, wp, wh;
  double t_submit, t_start, t_done;
  size_t footprint;           /* arena bytes the request held                 */
} edx_server_result;

void edx_server_default_opts(edx_server_opts* o);
edx_status edx_server_create(const edx_server_opts* opts, edx_server** out);
/* Queue a request (model arrays are copied); returns its ticket. */
edx_status edx_server_submit(edx_server* s, const edx_model* model, int32_t nup,
                             int32_t ndw, int64_t* ticket);
/* Result of a finished request (then forgotten by the server).  wait = 0
 * returns EDX_PENDING if it is not done.  g_out (nullable, host) receives
 * 2*lmats doubles. */
edx_status edx_server_poll(edx_server* s, int64_t ticket, int32_t wait,
                           edx_server_result* res, double* g_out);
edx_status edx_server_stats(edx_server* s, int32_t* pending, int32_t* running,
                            int64_t* completed, size_t* largest_free);
double edx_server_clock(void);
/* Waits for admitted requests, drops queued ones, frees the arena. */
void edx_server_destroy(edx_server* s);

const char* edx_status_str(edx_status st);
const char* edx_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* EDX_H */
