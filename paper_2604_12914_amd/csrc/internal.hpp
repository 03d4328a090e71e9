// Internal declarations of the lrcc library (not part of the ABI).
//
// Block-pair layout used by every kernel
// --------------------------------------
// Virtual indices are grouped in blocks of TB = 8; nbv = ceil(v / 8).  An
// ordered block pair (A, B) with A <= B has index
//   bp(A, B) = A * nbv - A * (A - 1) / 2 + (B - A),   nbp = nbv (nbv + 1) / 2,
// and holds NS = 64 slots s = a_l * 8 + b_l for a = 8A + a_l, b = 8B + b_l.
// A slot is live when a < b < v; dead slots hold zeros.
//
// Doubles (X, sigma, G) live on the device as planar arrays
//   buf[plane][bp][m][64],   m = r * o(o-1)/2 + ij,  m < Mp = roundup(M, 16)
// so the 64 slots of one block pair and all rows m form one contiguous run.
//
// Cholesky vectors are staged (once per call) as
//   Ls[A][C][P][plane][64],  64 = a_l * 8 + c_l,  P < ncp = roundup(nchol, KC)
// so one 8 x 8 block of every L^P is a contiguous 64-element run per plane.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/lrcc.h"

namespace lrcc {

constexpr int TB = 8;    // virtual indices per block
constexpr int NS = 64;   // slots per block pair
constexpr int WG = 256;  // threads per workgroup of the ladder kernels

inline long npair(long n) { return n * (n - 1) / 2; }
inline long roundup(long x, long m) { return (x + m - 1) / m * m; }

struct Geom {
  int o = 0, v = 0, nchol = 0, nrhs = 0;
  long npo = 0, npv = 0;  // occupied / virtual pair counts
  long M = 0, Mp = 0;     // rows (nrhs * npo) and rows padded to 16
  int nbv = 0, nbp = 0;   // virtual blocks, block pairs
  int ncp = 0;            // nchol padded to the chunk length
  long xb_plane() const { return (long)nbp * Mp * NS; }  // elements per plane
};

Geom make_geom(int o, int v, int nchol, int nrhs, int kc);

// Grow-only device buffer.
struct Buf {
  void* p = nullptr;
  size_t n = 0;
  hipError_t ensure(size_t bytes);
  void release();
  template <typename T> T* as() const { return static_cast<T*>(p); }
};

}  // namespace lrcc

struct lrcc_handle_s {
  int device = 0;
  hipStream_t stream = nullptr;
  std::string err;
  int ncu = 0;
  // ladder workspace
  lrcc::Buf ls, ls2;      // staged Cholesky vectors (ls2: second operand set)
  lrcc::Buf xb, sb, gb;   // block-layout doubles: input, accumulator, gradient
  lrcc::Buf tab;          // block-pair table
  lrcc::Buf hflag;        // nonzero when the staged L is not Hermitian (device int)
  lrcc::Buf order[3];     // tile order per precision (XCD-aware super-tiles), see tile_order()
  long order_key[3][6] = {{-1, -1, -1, -1, -1, -1}, {-1, -1, -1, -1, -1, -1},
                          {-1, -1, -1, -1, -1, -1}};
  int order_s[3] = {0, 0, 0};  // super-tile width per precision (0 = default)
  int occ[3][2] = {};     // launch variant per precision and complex form (0 = default)
  lrcc::Buf vws;          // bf16x3: one panel of antisymmetrised integral tiles
  lrcc::Buf bitems;       // bf16x3: build items of every panel (int2), see build_items()
  std::vector<long> bitems_key, bitems_off;  // their geometry key and per-panel offsets
  size_t panel_cap = 0;   // bytes allowed for vws (0 = not yet chosen)
  int tab_nbv = -1;
  int deterministic = 0;  // ladders without atomics, reproducible bit for bit (lrcc_set_deterministic)
  // solver workspace
  lrcc::Buf sv[12];
  lrcc::Buf hw;           // hole-hole ladder: W matrix and occupied pair table
  lrcc::Buf cw;           // pivoted Cholesky: remaining diagonal and state
  lrcc::Buf fw;           // FNS++ and eigensolver workspace
  lrcc::Buf rw;           // ring term workspace
  void* rb = nullptr;     // rocBLAS handle (gradient GEMMs), created on first use
  // ladder-kernel timing (lrcc_set_timing)
  bool timing = false;
  std::vector<hipEvent_t> tev;  // start/stop pairs
  size_t tev_used = 0;          // pairs recorded since enabling
};

namespace lrcc {

// Status helpers -------------------------------------------------------------
lrcc_status fail(lrcc_handle h, lrcc_status s, const std::string& msg);
lrcc_status hip_fail(lrcc_handle h, hipError_t e, const char* what);

#define LRCC_HIP(h, call)                                   \
  do {                                                      \
    hipError_t e_ = (call);                                 \
    if (e_ != hipSuccess) return ::lrcc::hip_fail(h, e_, #call); \
  } while (0)

// Staging / layout launchers (layout.hip) ----------------------------------
// Which matrix of each L^P the staging writes: L^P itself, its conjugate
// transpose (the adjoint ladder) or its transpose (the ladder's transpose,
// for the left-hand response: K(L^T) = K(L)^T).
enum LForm { L_PLAIN = 0, L_ADJ = 1, L_TRANS = 2 };
// Stage L (complex, dtype dt) into planar blocks of type T, planes (re, im)
// (both complex forms read these), in the form `form`.
template <typename T>
hipError_t stage_L(const void* L, lrcc_dtype dt, const Geom& g, LForm form, T* Ls,
                   hipStream_t st);
// Packed doubles -> planar block layout (2 planes of T); dead slots and pad
// rows are written as zero.
template <typename T>
hipError_t pack_to_block(const void* X, lrcc_dtype dt, const Geom& g,
                         const int* tab, T* Xb, hipStream_t st);
// Planar block layout (2 planes of T) -> packed doubles in dtype dt.
template <typename T>
hipError_t block_to_pack(const T* Sb, const Geom& g, const int* tab, void* S,
                         lrcc_dtype dt, hipStream_t st);
hipError_t fill_zero(void* p, size_t bytes, hipStream_t st);
// nonherm[0] = 0 if every L^P is exactly Hermitian (L^P_ca == conj L^P_ac,
// compared bit for bit after conversion to double), 1 otherwise.  nonherm
// must point to at least 16 bytes; it is cleared here with a fill kernel.
hipError_t herm_check(const void* L, lrcc_dtype dt, int v, int nchol, int* nonherm,
                      hipStream_t st);

// Ladder launchers (ppl_mfma.hip) -------------------------------------------
// Sb (2 planes, accumulated with atomics) += PPL of Xb.  One workgroup per
// tile pair (ab, cd) with ab <= cd (ppl_ntile of them, listed by `order`),
// which also covers the mirror (cd, ab); *nonherm (device) selects whether
// the mirror reuses the tile (Hermitian L) or is built.  Sb must be zeroed
// by the caller.
long ppl_ntile(const Geom& g);
hipError_t ppl_launch(lrcc_prec prec, lrcc_cmul cmul, bool acc64, const Geom& g,
                      const void* Ls, const void* Xb, void* Sb, const int* tab,
                      const int* order, const int* nonherm, int occ, hipStream_t st);
// One instance of the persistent FP64 ladder (k_ppl_queue): its staged
// vectors, block-layout doubles and accumulator, geometry, tile order and
// the first queue item that belongs to it.
// Items of instance i: local index l < 2 ppl_ntile (tiles, then mirrors).
// The queue has one counter per XCD; XCD x owns the items l = x (mod nx) of
// every instance, in instance order, and xstart[x] is the number of them in
// the instances before this one.
constexpr int QXMAX = 8;  // XCDs tracked by the queue
struct BatchInst {
  const double* Ls;
  const double* Xb;
  double* Sb;
  const int* tab;
  const int* order;    // ppl_ntile tile pairs ab <= cd (XCD-aware super-tile order)
  const int* nonherm;  // device flag of this instance's L
  int nbv, nbp, ncp, Mp, v;
  long start;              // first item in a single global list
  long xstart[QXMAX];      // first item in each XCD's list
};
// counter: nx (<= QXMAX) zeroed unsigned counters; xtotal[x]: items of XCD x;
// cm3: the 3M complex form (same staged layout as 4M).
hipError_t ppl_queue_launch(const BatchInst* inst, int ninst, const long* xtotal, int nx,
                            unsigned* counter, int nwg, bool cm3, hipStream_t st);
// Deterministic ladder (no atomics; one workgroup per block pair AB owning
// sigma[:, AB], every tile built in ascending CD order, 4M form): Sb zeroed
// by the caller; FP64 or FP32 arithmetic on the ppl_launch staged layouts.
hipError_t ppl_det_launch(lrcc_prec prec, bool acc64, const Geom& g, const void* Ls,
                          const void* Xb, void* Sb, const int* tab, hipStream_t st);
int ppl_chunk(lrcc_prec prec, lrcc_cmul cmul);   // KC of the staged layout
bool ppl_has_variant(lrcc_prec prec, lrcc_cmul cmul, int variant);  // 4M launch variants 1-5
size_t ppl_ls_bytes(lrcc_prec prec, lrcc_cmul cmul, const Geom& g);
size_t ppl_xb_bytes(lrcc_prec prec, const Geom& g);

// ppl_launch on the handle's stream, bracketed by timing events when the
// handle has timing enabled.
lrcc_status ppl_run(lrcc_handle h, lrcc_prec prec, lrcc_cmul cmul, bool acc64, const Geom& g,
                    const void* Ls, const void* Xb, void* Sb, const int* nonherm);

// Pivoted Cholesky decomposition (chol.hip) ----------------------------------
// Workspace bytes for n rows; run the decomposition of M (n x n complex128,
// device) into L [maxv][n] (device) with optional pivots [maxv] (device);
// *nvec (host) receives the vector count.  Synchronous on st.
size_t chol_state_bytes(long n);
hipError_t chol_run(long n, const void* M, double tau, int maxv, void* L, int* pivots, void* ws,
                    int* nvec, hipStream_t st);

// Hermitian eigensolver (heev.hip) -------------------------------------------
// Workspace bytes for an n x n problem; eigenpairs of A (n x n complex128,
// row-major, device, not modified): w[n] (device) ordered ascending (mode 0)
// or by descending magnitude (mode 1), the first ncol_out eigenvectors as
// columns of Vout [n][ncol_out] (device; may be NULL), the ordering
// permutation in perm_out (device; may be NULL).  The unordered eigenvectors
// stay in the workspace (heev_vectors) until its next use.  Synchronises st
// once per sweep; *sweeps (host, may be NULL) gets the sweep count.
size_t heev_ws_bytes(int n);
hipError_t heev_run(int n, const void* A, int mode, double* w, void* Vout, int ncol_out,
                    void* ws, int* perm_out, int* sweeps, hipStream_t st);
const void* heev_vectors(const void* ws, int n);
// Out[r][k] = V[r][perm[k]], k < ncol (row stride ncol); Sout (if not NULL)
// = diag(scale) Out.
hipError_t gather_cols(int n, int ncol, const void* V, const int* perm, void* Out,
                       const double* scale, void* Sout, hipStream_t st);

// FNS++ natural spinors (fns.hip) ---------------------------------------------
size_t fns_ws_bytes(int o, int v, int ncomp);
lrcc_status fns_run(lrcc_handle h, int o, int v, int nchol, const double* eps, const void* Lov,
                    int ncomp, const void* Aov, const void* Avv, const void* Aoo, double omega,
                    double threshold, double* occ, void* B, double* eps_new, int* keep,
                    void* gamma, double* hbar_out, void* ws, lrcc_fns_info* info);
size_t fns_transform_ws_bytes(int v, int k, int nchol);
lrcc_status fns_transform(lrcc_handle h, int v, int k, int nchol, int nrow, const void* B,
                          const void* L, const void* mu, void* Lt, void* mut, void* ws);

// Ring term (ring.hip) --------------------------------------------------------
// sigma (+)= P(ij)P(ab) sum_kc <kb||cj> X_ik^ac on packed complex128 doubles.
size_t ring_ws_bytes(int o, int v, int nrhs);
// The particle-hole integral matrix M[(kc)][(jb)] = <kb||cj> ((o v)^2
// complex), from the blocks of L^P or, with `transposed`, of (L^P)^T (the
// transposed operator, for the left-hand solve); and its application to
// packed doubles (workspace sizes below).
size_t ring_m_bytes(int o, int v);
size_t ring_build_ws_bytes(int o, int v, int nchol, bool transposed);
size_t ring_apply_ws_bytes(int o, int v, int nrhs);
lrcc_status ring_build_m(lrcc_handle h, int o, int v, int nchol, const void* Loo,
                         const void* Lov, const void* Lvo, const void* Lvv, bool transposed,
                         double2* M, void* ws);
lrcc_status ring_apply(lrcc_handle h, int o, int v, int nrhs, const double2* M, const void* X,
                       void* S, bool accumulate, void* ws);
lrcc_status ring_run(lrcc_handle h, int o, int v, int nchol, int nrhs, const void* Loo,
                     const void* Lov, const void* Lvo, const void* Lvv, const void* X, void* S,
                     bool accumulate, void* ws);

// Hole-hole ladder (hhl.hip) ------------------------------------------------
// W[(ij),(kl)] = scale <kl||ij> from occupied-occupied vectors Loo [nchol][o][o]
// (dtype dt; form L_TRANS: from (L^P)^T, which gives W^T); otab[p] = (i<<16)|j
// of packed occupied pair p (device).  W: npo*npo complex (device).  scale 2:
// the hole-hole ladder with the unrestricted k, l sum; 1: half of it, as the
// T = 0 doubles-doubles block of the model Jacobian holds it.
hipError_t hh_build_w(const void* Loo, lrcc_dtype dt, int o, int nchol, const int* otab,
                      LForm form, double scale, double2* W, hipStream_t st);
// otab[p] = (i << 16) | j of the packed occupied pairs (device, npo ints).
hipError_t hh_pair_table(int o, int* otab, hipStream_t st);
// Sb += W X per block pair and right-hand side on the block layout (FP64
// planes re, im); Xb and Sb as the ladder's.
hipError_t hh_apply(const double2* W, const Geom& g, const double* Xb, double* Sb,
                    hipStream_t st);

// bf16x3 ladder (ppl_bf16x3.hip): staged layouts and the panel driver.
int bf16x3_chunk();
size_t bf16x3_ls_bytes(const Geom& g);
size_t bf16x3_xb_bytes(const Geom& g);
// Panel rows [ab0, ab0 + n): upper tiles, and bytes with their mirrors.
long bf16x3_panel_tiles(const Geom& g, int ab0, int n);
size_t bf16x3_panel_bytes(const Geom& g, int ab0, int n);
hipError_t bf16x3_stage_L(const void* L, lrcc_dtype dt, const Geom& g, LForm form, void* Ls,
                          hipStream_t st);
hipError_t bf16x3_pack_x(const void* X, lrcc_dtype dt, const Geom& g, const int* tab, void* Xb,
                         hipStream_t st);
hipError_t bf16x3_split_x(const double* x, const Geom& g, void* Xb, hipStream_t st);
// Panels of at most `cap` bytes (at least one row each) in Vws; Sb zeroed by
// the caller; *nonherm (device) as for ppl_launch.
hipError_t bf16x3_run(lrcc_handle h, const Geom& g, const void* Ls, const void* Xb, void* Sb,
                      bool acc64, void* Vws, size_t cap, const int* tab, const int* nonherm,
                      hipStream_t st);
// Run the bf16x3 ladder with the handle's panel workspace (sized here).
lrcc_status bf16x3_apply(lrcc_handle h, const Geom& g, const void* Ls, const void* Xb, void* Sb,
                         bool acc64, const int* nonherm);

// dL = gradient of sigma with respect to L (ppl_grad.hip); packed X, G.
lrcc_status grad_L(lrcc_handle h, const Geom& g, const void* L, const void* X, const void* G,
                   void* dL, lrcc_dtype dt);

// Tile order for a launch over AB block pairs [ab0, ab1) x all CD (upper:
// only CD >= AB): entry w is the tile (ab - ab0) * nbp + cd run by workgroup
// w.  Tiles are grouped
// into super-tiles whose AB and CD pairs come from s-wide ranges of virtual
// blocks (so the four Cholesky blocks a tile reads fall in s x s sets), and
// each XCD receives a contiguous run of super-tiles (workgroups go to XCDs
// round-robin).  Returns a device pointer owned by the handle.
const int* tile_order(lrcc_handle h, const Geom& g, int ab0, int ab1, bool upper,
                      lrcc_prec prec, lrcc_status* st);

// Host-side builders of the block-pair table and of the super-tile order
// (nx = number of XCDs to split the order over; 1 = plain super-tile order).
void block_pair_table(int nbv, std::vector<int>* tab);
void supertile_order(const Geom& g, int ab0, int ab1, int sw, int nx, bool upper,
                     std::vector<int>* ord);

// Autotuner (tune.hip); arguments already validated.
lrcc_status autotune_impl(lrcc_handle h, int o, int v, int nchol, int nrhs, lrcc_prec prec,
                          lrcc_cmul cmul, const char* cache_path, lrcc_tune_result* out);

// Batched solve (solver.hip); arguments already validated.
lrcc_status solve_batched_impl(lrcc_handle h, int ninst, const lrcc_instance* inst,
                               const lrcc_solve_opts* opts, lrcc_solve_info* info);

// Block-pair table: tab[bp] = (A << 16) | B.
lrcc_status ensure_tab(lrcc_handle h, int nbv);

// Full sigma on device pointers in the packed layout (used by the API and
// the solver).  X, S packed in dtype dt.
lrcc_status sigma_packed(lrcc_handle h, const Geom& g, const void* L, bool conj_t,
                         const void* X, void* S, lrcc_dtype dt, lrcc_prec prec,
                         lrcc_cmul cmul);

// Allocation-free ladder (noalloc.hip): the per-device address of the static
// scratch array is looked up by noalloc_init (called by lrcc_create with the
// device current); sigma_noalloc runs the FP64 / FP32 ladder in it.
void noalloc_init(int device);
size_t noalloc_scratch_bytes();
lrcc_status sigma_noalloc(lrcc_handle h, const Geom& g, const void* L, const void* X, void* S,
                          lrcc_dtype dt, lrcc_prec prec, lrcc_cmul cmul);

// Response solve (solver.hip); arguments already validated.
lrcc_status solve_impl(lrcc_handle h, int o, int v, int nchol, const double* eps, const void* L,
                       int ncomp, const void* mu, int nomega, const double* omegas,
                       const lrcc_solve_opts* opts, double* alpha, lrcc_solve_info* info);

}  // namespace lrcc
