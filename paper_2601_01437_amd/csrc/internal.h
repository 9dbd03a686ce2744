// Internal declarations of the gfx950 LM-operator library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "irlnqs.h"

namespace irl {

constexpr int kMaxKrylov = 64;          // m <= 64
constexpr int kMaxBlock = 8;            // vectors per multi-vector apply / block Lanczos step
constexpr int kBasisCols = kMaxKrylov + kMaxBlock;   // Krylov basis columns held per buffer
constexpr int kCheckStride = 1;         // Lanczos steps between in-cycle convergence tests (large operators)
constexpr int kWave = 64;               // CDNA wavefront width
constexpr int kStreamBlocks = 512;      // row blocks of the D~^T stream kernel
constexpr int kMaxColBlocks = 8;        // column blocks of stored Hamiltonian rows
constexpr int64_t kColSliceBytes = 2 << 20;   // w bytes per column block (an L2 share)
constexpr int kReduceGroups = 16;       // first-level groups of the partial reduction
constexpr int kScalarParts = 1024;      // blocks of the scalar (energy) reductions
constexpr uint64_t kEmptyKey = ~0ull;   // empty hash slot
// fixed device scratch of irl_lookup_noalloc: staged keys (8 B) and rows (4 B)
constexpr int64_t kNoAllocMaxKeys = 1 << 18;
constexpr size_t kNoAllocScratchBytes = (size_t)kNoAllocMaxKeys * 12;

// Device scalars kept in the first bytes of a workspace.
struct WsScalars {
    double Z;            // psi^T psi
    double E_el;         // psi^T H psi / Z (electronic)
    double sum_psi2[2];  // compensated (sum, compensation)
    double sum_psih[2];
    double resid2;       // squared norm of an explicit residual
    double rnorm;        // scratch norm
    double normT;        // running max |alpha|, |beta| of the current T
    double lam;          // selected Ritz value
    double resid_est;    // |beta_m u_1[m-1]|
    double gap;
    double c0;
    int32_t breakdowns;  // Lanczos breakdowns in the current solve
    int32_t restarts;    // implicit restarts done in the current solve (seeds derive from it)
    double alpha[kMaxKrylov];
    double beta[kMaxKrylov];
    double ritz[kMaxKrylov];
    double talpha[kMaxKrylov];   // T after restart (leading k)
    double tbeta[kMaxKrylov];
    double Q[kMaxKrylov * kMaxKrylov];   // restart rotations, column-major Q[l + m*i]
    double U[kMaxKrylov * kMaxKrylov];   // Ritz vectors of T, column-major
    double h[kMaxKrylov + 1];            // Gram-Schmidt coefficients
    // block Lanczos: projected matrix T = Q^T H~' Q over the basis and the next
    // block (row-major, leading dimension kBasisCols)
    double T[kBasisCols * kBasisCols];
};

// Workspace layout for one (N_s, ncols, flags).
struct WsLayout {
    int64_t ns = 0, ncols = 0;
    int64_t ld64 = 0, ld32 = 0, ldv = 0;   // row strides (elements) and vector length
    uint32_t flags = 0;
    size_t off_scal = 0, off_d64 = 0, off_d32 = 0, off_psi = 0, off_hpsi = 0, off_w = 0,
           off_u = 0, off_grad = 0, off_yh = 0, off_ys = 0, off_y = 0, off_r = 0,
           off_part = 0, off_part2 = 0, off_red = 0, off_kry0 = 0, off_kry1 = 0, off_vconv = 0,
           off_img0 = 0, off_img1 = 0, off_hy = 0,   // operator images of the basis; of y
           off_fac = 0,                              // factored Jacobian d = 1 - t^2 (N_s x hfac)
           off_sig = 0,                              // D~^T psi (connected basis, mode C)
           off_q = 0,                                // sampled row weights Z c_r / (N psi_r^2)
           off_warm = 0,                             // Ritz vector of the last converged solve
           // drawn rows gathered contiguously (IRL_WS_SAMPLED with the factored Jacobian)
           off_ckeys = 0, off_cpsi = 0, off_cq = 0, off_cel = 0, off_crow = 0, off_cfac = 0;
    int hfac = 0;                                    // hidden units of the factored Jacobian
    int kf_S = 0;   // alpha ranges of the full-space backward product (0: the matrix-core kernel)
    size_t total = 0;
};

// V: visible units (2 n_orb); with IRL_WS_FACTORED the hidden width follows from
// ncols = V H + H + V + 1 (hfac = 0 when ncols fits no network)
// fullA, fullB: string counts of a full space (0 otherwise), which enable the
// string-split backward product of the factored Jacobian
WsLayout make_layout(int64_t ns, int64_t ncols, uint32_t flags, int V, int64_t fullA = 0, int64_t fullB = 0);

// Full-space backward product of the factored Jacobian: alpha ranges S (0 when the
// product keeps the matrix-core kernel)
int fac_full_ranges(int64_t nA, int64_t nB, int n, int H);

// vectors the w/u, yH/yS and conversion regions of a layout hold (1, or kMaxBlock with IRL_WS_BLOCK)
inline int layout_vectors(const WsLayout &L) { return (L.flags & IRL_WS_BLOCK) ? kMaxBlock : 1; }

template <typename T>
inline T *ws_ptr(void *ws, size_t off) { return reinterpret_cast<T *>(static_cast<char *>(ws) + off); }

// Device tables owned by a system handle.
struct SystemDev {
    uint64_t *keys = nullptr;   // ascending, n_dets
    double *h = nullptr;        // n*n
    double *g = nullptr;        // n^4
    double *diag = nullptr;     // n_dets
    // hashed lookup (any set)
    uint64_t *hkeys = nullptr;  // capacity
    int32_t *hrows = nullptr;   // capacity
    uint64_t hcap = 0;
    uint32_t *hfilter = nullptr;  // membership bitmap, 2^hfbits bits, indexed by the top hash bits
    int hfbits = 0;
    // blocked lookup (selected sets, n <= 24): rows sharing a beta string are contiguous
    int32_t *bidx = nullptr;      // 2^n: beta string -> block index, -1 if absent
    int32_t *bstart = nullptr;    // nblocks + 1 row offsets
    int64_t nblocks = 0;
    // the same rows alpha-major: rows sharing an alpha string, in beta order
    int32_t *aidx = nullptr;      // 2^n: alpha string -> alpha block index, -1 if absent
    int32_t *astart = nullptr;    // alpha blocks + 1 offsets into arow / abeta
    int32_t *arow = nullptr;      // n_dets rows in alpha-major order
    uint32_t *abeta = nullptr;    // their beta strings
    // stored rows (optional): off-diagonal elements inside the set, compressed by row
    int64_t *hptr = nullptr;      // hcb blocks of n_dets + 1 row offsets (block-major)
    int32_t *hcol = nullptr;      // nnz target rows, block b's targets in [b 2^hcs, (b + 1) 2^hcs)
    double *hval = nullptr;       // nnz values
    int64_t hnnz = 0;
    int32_t hcb = 0;              // column blocks of the stored rows
    int32_t hcs = 0;              // log2 of the target rows per column block
    // stored rows, LDS-sliced layout (large sets): column slices of 2^scs target rows
    // (a slice of w staged in LDS); per slice, rows in windows of kSellWindow ordered
    // by element count and grouped 64 per wavefront, group g holding glen[g] x 64
    // slots (slot (j, lane): the lane row's j-th element, zero padding past its end)
    int64_t *sbase = nullptr;     // scb slot offsets of the slices
    uint32_t *sgbase = nullptr;   // scb x sgroups slot offsets of the groups (inside the slice)
    uint16_t *sglen = nullptr;    // scb x sgroups slots per lane of the groups
    uint16_t *sperm = nullptr;    // scb x sgroups x 64: row of each lane inside its window (0xffff: none)
    uint16_t *scol = nullptr;     // slots: targets (row - slice start)
    double *sval = nullptr;       // slots: values
    double *spart = nullptr;      // scb x n_dets partial sums of one apply
    int64_t sslots = 0;           // slots, padding included
    int32_t sgroups = 0;          // ceil(n_dets / 64)
    int32_t scb = 0;              // slices (0: the L2-block layout above, if any)
    int32_t scs = 0;
    // string tables (full space)
    int32_t *rankA = nullptr;   // 2^n, -1 for strings not of popcount n_alpha
    int32_t *rankB = nullptr;
    uint32_t *strA = nullptr;   // alpha strings by rank
    uint32_t *strB = nullptr;
    // product-kernel tables (full space)
    uint32_t *sglA = nullptr;   // nA x (na*va): rank<<10 | sign<<9 | i<<5 | a
    uint32_t *sglB = nullptr;
    uint16_t *sglA_ia = nullptr;
    uint16_t *sglB_ia = nullptr;
    double *jB = nullptr;
    double *fA = nullptr;       // nA x (na*va): h_ia + sum_{j in alpha}[(ia|jj)-(ij|ja)]
    double *fB = nullptr;
    int32_t *dblA_rank = nullptr;   // nA x (C(na,2) C(va,2))
    double *dblA_val = nullptr;
    int32_t *dblB_rank = nullptr;
    double *dblB_val = nullptr;
    double *jA = nullptr;       // nA x n*n: sum_{i in alpha} (pq|ii)
    double *denseA = nullptr;   // nA x nA same-spin alpha doubles as a dense symmetric matrix (or nullptr)
    double *denseB = nullptr;   // nB x nB, beta
};

// Read-only view of a system's Hamiltonian tables (pull kernels, solo and grouped).
struct HamView {
    int n, na, nb, full;
    int64_t ns, nA;
    const uint64_t *keys;
    const double *diag, *h, *g;
    const uint64_t *hkeys;
    const int32_t *hrows;
    uint64_t hmask;
    const uint32_t *hfilter;
    int hfbits;
    const int32_t *rankA, *rankB;
    const int32_t *bidx;     // blocked lookup: beta string -> block, -1 if absent (or nullptr)
    const int32_t *bstart;   // blocked lookup: first row of each block, plus the end
    const int32_t *aidx;     // blocked lookup: alpha string -> alpha block, -1 if absent
    const int32_t *astart;   // blocked lookup: alpha blocks' offsets into arow / abeta
    const int32_t *arow;     // blocked lookup: rows in alpha-major order
    const uint32_t *abeta;   // blocked lookup: their beta strings
    const int64_t *hptr;     // stored rows (or nullptr): row offsets, hcb blocks of ns + 1
    const int32_t *hcol;     // stored rows: targets
    const double *hval;      // stored rows: values
    int hcb, hcs;            // stored rows: column blocks, log2 of their width in rows
    const int64_t *sbase;    // stored rows, LDS-sliced layout (or nullptr)
    const uint32_t *sgbase;
    const uint16_t *sglen, *sperm, *scol;
    const double *sval;
    double *spart;           // stored rows, LDS-sliced layout: per-slice partial sums of an apply
    int scb, scs, sgroups;
};

// key -> row lookup used when excitations are enumerated
enum LookupMode { kLkRanks = 0, kLkHash = 1, kLkBlocks = 2 };

// One member of a grouped (batched) launch: its system view, workspace
// pointers and network.  Lives in device memory; grouped kernels index it.
struct Member {
    HamView ham;
    const double *D64;
    const float *D32;
    int64_t ld, ncols, ns;
    double *psi, *hpsi, *w, *u, *grad, *yH, *yS, *y, *r, *part, *part2, *red, *vconv;
    double *kry[2];
    double *img[2];   // operator images of the basis vectors
    double *hy;       // operator image of the Ritz vector
    WsScalars *sc;
    int32_t V, H;
    double *theta;
    double *dtheta;
    int32_t nblk_t2;     // row blocks of the D~^T stream (same as the solo launch)
    int32_t nparts_e;    // blocks of the energy reduction (same as the solo launch)
};

// A unit of grouped work: member m, kernel-specific indices a, b, rows [r0, r1).
struct WorkItem {
    int32_t m, a, b, pad;
    int64_t r0, r1;
};

// Scalars gathered from every member after a grouped phase (one readback).
struct MemberScalars {
    double Z, E_el, lam, resid_est, gap, normT, c0, resid2;
};

}  // namespace irl

struct irl_system {
    int32_t n = 0, na = 0, nb = 0;
    double e_core = 0.0;
    int64_t ns = 0;
    int64_t nA = 0, nB = 0;   // string counts (full space) or distinct counts
    bool full = false;
    uint32_t sys_flags = 0;   // irl_system_flags given at create
    int ham_kernel = 0;       // 0 hashed pull, 1 rank pull, 2 string product, 3 blocked pull,
                              // 4 stored rows
    int lookup = 0;           // irl::LookupMode of the excitation enumeration
    // launch shapes set by irl_tune_set (0: the built-in default); both only move
    // rows between workgroups, so results do not depend on them
    int32_t tune_lut_blocks = 0;    // workgroups of the table-driven forward pass and D~ v
    int32_t tune_pull_blocks = 0;   // workgroup cap of the enumerating Hamiltonian apply
    int32_t tune_pull_waves = 0;    // wavefronts (rows) per workgroup of that apply: 1, 2 or 4
    int device = 0;
    size_t dev_bytes = 0;
    irl::SystemDev d;
    std::string err;
    // last workspace evaluated into
    void *ws = nullptr;
    irl::WsLayout lay;
    bool ws_valid = false;
    bool ws_has64 = false, ws_has32 = false;
    double Z = 0.0, E_el = 0.0;   // host copies after the last evaluation
    // the last converged single-vector solve (IRL_STEP_WARM_START): its workspace,
    // dimension, mode and the offset of the copy of its Ritz vector in that workspace
    void *warm_ws = nullptr;
    int64_t warm_ncols = 0;
    size_t warm_off = 0;
    int warm_mode = -1;
    // sampled estimators (irl_vmc_sample) replace the exact ones until the next evaluation
    bool vmc = false;
    double E_exact = 0.0;
    int64_t vmc_rows = 0;     // drawn rows gathered contiguously (0: products run over every row)
    // pinned host staging for small readbacks
    irl::WsScalars *host_scal = nullptr;
    // captured Lanczos cycles (graph replay of small operators); owned by api.hip
    void *cycle_graphs = nullptr;
    hipStream_t capture_stream = nullptr;
    // per-kernel timing
    bool stats_on = false;
    bool ev_open = false;           // stat_begin recorded the first event of a pair
    uint32_t stat_mask = (1u << IRL_STAT_KINDS) - 1u;   // kinds that get events
    std::vector<hipEvent_t> ev_pool;
    std::vector<int> ev_kind;       // kind of pending pair i (events 2i, 2i+1)
    size_t ev_used = 0;
    double stat_ms[IRL_STAT_KINDS] = {0};
    int64_t stat_cnt[IRL_STAT_KINDS] = {0};
};

namespace irl {

// ---- kernels (launch wrappers; all enqueue on `st`) ----
// system.hip
hipError_t launch_enumerate_full(uint64_t *keys, uint32_t *strA, uint32_t *strB, int32_t *rankA,
                                 int32_t *rankB, int n, int na, int nb, int64_t nA, int64_t nB,
                                 hipStream_t st);
hipError_t launch_hash_build(const uint64_t *keys, int64_t ns, uint64_t *hkeys, int32_t *hrows,
                             uint64_t cap, uint32_t *filter, int fbits, hipStream_t st);
hipError_t launch_hash_lookup(const uint64_t *hkeys, const int32_t *hrows, uint64_t cap,
                              const uint64_t *q, int64_t nq, int32_t *rows, hipStream_t st);
hipError_t launch_diagonal(const uint64_t *keys, int64_t ns, int n, const double *h,
                           const double *g, double *diag, hipStream_t st);
// fixed scratch (system.hip): resolve the device address of the array once per
// device (with that device current at the call), then return it (nullptr before)
hipError_t noalloc_scratch_setup(int device);
void *noalloc_scratch(int device);
// stored rows, LDS-sliced layout (hamiltonian.hip): count[b n_dets + row] = connections of
// row inside slice b; fill writes them to the slots of (slice b, lane slot[b][row] =
// group * 64 + lane), element j of the row at slot base + j * 64 + lane, in the
// lane-major enumeration order of its wavefront
#ifndef IRL_SLICE_LOG
#define IRL_SLICE_LOG 14
#endif
constexpr int kSliceLog = IRL_SLICE_LOG; // 2^14 target rows (128 KiB of w) per slice
constexpr int kMaxSlices = 256;          // sets of up to 2^22 determinants
constexpr int kSellWindow = 4096;        // rows ordered by length together
hipError_t launch_ham_count_sliced(const irl_system *s, int scs, int scb, uint32_t *count, hipStream_t st);
hipError_t launch_ham_fill_sliced(const irl_system *s, int scs, int scb, const uint32_t *slot, uint16_t *scol,
                                  double *sval, hipStream_t st);
hipError_t launch_lookup_any(const irl_system *s, const uint64_t *q, int64_t nq, int32_t *rows,
                             hipStream_t st);

// hamiltonian.hip
hipError_t launch_product_tables(irl_system *s, hipStream_t st);
// release the dense doubles and their BLAS handle
void free_dense_doubles(irl_system *s);
HamView ham_view(const irl_system *s);
hipError_t launch_ham_stored_grouped(const Member *M, const WorkItem *items, int nitems,
                                     int64_t nblocks, int which, hipStream_t st);
// max_n: the largest orbital count among the members the items cover
hipError_t launch_ham_pull_grouped(const Member *M, const WorkItem *items, int nitems,
                                   int64_t nblocks, int which, int lookup, int max_n, hipStream_t st);
hipError_t launch_ham_apply(const irl_system *s, const double *w, double *u, hipStream_t st);
// rows [r0, r1) of u = H w (r0, r1 multiples of ham_row_quantum: whole beta strings
// for the string-product kernel)
hipError_t launch_ham_apply_rows(const irl_system *s, const double *w, double *u, int64_t r0, int64_t r1,
                                 hipStream_t st);
int64_t ham_row_quantum(const irl_system *s);
// multi-vector D~ streams: W[:, q] = D~ V[:, q] (q < nb, W column stride ns) and the
// 2 nb right-hand-side D~^T pass over (W, U); reduction into YS[:, q], YH[:, q] (stride ldy)
hipError_t launch_gemv_rows_multi(const WsLayout &L, void *ws, int prec, const double *V, int64_t ldv_in,
                                  int nb, int zero_v0, double *W, hipStream_t st);
hipError_t launch_gemv_t2_multi(const WsLayout &L, void *ws, int prec, int nb, const double *W,
                                const double *U, int *nblk, hipStream_t st);
hipError_t launch_t2_reduce_multi(const WsLayout &L, void *ws, int nblk, int nb, double *YS, double *YH,
                                  int64_t ldy, hipStream_t st);
// block Lanczos (one workgroup each): start block, step, Ritz pairs of T, thick restart
hipError_t launch_block_start(const WsLayout &L, void *ws, double *V, int nb, int mode, uint64_t seed,
                              hipStream_t st);
hipError_t launch_block_step(const WsLayout &L, void *ws, double *V, double *img, int s0, int nb, int mode,
                             int split, uint64_t seed, hipStream_t st);
hipError_t launch_block_ritz(const WsLayout &L, void *ws, int s, int nb, hipStream_t st);
hipError_t launch_block_restart(const WsLayout &L, void *ws, const double *Vold, double *Vnew,
                                const double *Iold, double *Inew, int s, int k, int nb, hipStream_t st);
// stored rows: per-row counts of connections inside the set, then the fill
// per column block b: count[b n_dets + row] = elements of row with targets in block b
hipError_t launch_ham_count(const irl_system *s, int32_t *count, hipStream_t st);
hipError_t launch_ham_fill(const irl_system *s, const int64_t *ptr, int32_t *col, double *val,
                           hipStream_t st);
hipError_t launch_ham_row_list(const irl_system *s, int64_t row, int32_t *tgt, int8_t *sign,
                               uint8_t *kind, double *val, int32_t *count, int cap,
                               hipStream_t st);

// nqs.hip
// FP64 D~^T (H psi - E psi) recomputed from theta into the D~^T partial rows (nblk row blocks)
hipError_t launch_nqs_grad(const irl_system *s, int V, int H, const double *theta, const WsLayout &L,
                           void *ws, int nblk, hipStream_t st);
// factored Jacobian: w = D~ v and partial rows of D~^T (y - coef psi) (half 0 or 1)
hipError_t launch_fac_forward(const irl_system *s, const WsLayout &L, void *ws, const double *theta,
                              hipStream_t st);
hipError_t launch_fac_jvp(const irl_system *s, const WsLayout &L, void *ws, const double *v, int zero_v0,
                          double *w, hipStream_t st);
// D~^T c into the partial rows: one right-hand side y0 (c = y0 - coef psi) into half
// `half`, or two (y1 non-null: y0 into half 0, y1 into half 1) from one pass over d
hipError_t launch_fac_vjp(const irl_system *s, const WsLayout &L, void *ws, const double *y0, const double *y1,
                          const double *coefp, int half, int nblk, hipStream_t st);
int fac_row_blocks(const irl_system *s, const WsLayout &L);
// the same products over an explicit row set (keys, psi and d of ns rows), e.g. the
// drawn rows of a sampled step gathered contiguously
struct FacRows {
    const uint64_t *keys;
    int64_t ns;
    const double *psi;
    const double *dfac;
};
hipError_t launch_fac_jvp_rows(const irl_system *s, const WsLayout &L, const FacRows &R, const double *v,
                               int zero_v0, double *w, hipStream_t st);
hipError_t launch_fac_vjp_rows(const irl_system *s, const WsLayout &L, void *ws, const FacRows &R,
                               const double *y0, const double *y1, const double *coefp, int half, int nblk,
                               hipStream_t st);
int fac_row_blocks_n(const irl_system *s, int64_t ns, int hfac);
// partial rows left by launch_fac_vjp over every row of ws
int fac_vjp_blocks(const irl_system *s, const WsLayout &L);
// 1 when D~ v on `ns` rows of this system with hidden width H runs the
// table-driven kernel (the one IRL_TUNE_LUT_BLOCKS shapes)
int fac_jvp_uses_lut(const irl_system *s, int64_t ns, int H);
hipError_t launch_nqs_dtilde(const irl_system *s, int V, int H, const double *theta,
                             const WsLayout &L, void *ws, hipStream_t st);
hipError_t launch_dtilde_import(const void *D, int64_t ld, int64_t ncols, int dtype,
                                const WsLayout &L, void *ws, hipStream_t st);

// dtilde.hip
// zero_v0: treat v[0] as zero (split form: the psi column is handled in FP64 through g)
hipError_t launch_gemv_rows(const WsLayout &L, void *ws, int prec, const double *v, double *w,
                            int zero_v0, hipStream_t st);
// [yS, yH] = D~^T [a, b] where a = w (or nullptr), b = u - scale*psi form; see dtilde.hip
// stream part: per-row-block partial sums; returns the number of row blocks
// the D~^T launch restricted to its row blocks [rbA, rbB) (same partials as the full launch)
hipError_t launch_gemv_t2_blocks(const WsLayout &L, void *ws, int prec, const double *a,
                                 const double *b, const double *b_sub, const double *b_coef,
                                 int *nblk, int rbA, int rbB, hipStream_t st);
int gemv_t2_row_blocks(const WsLayout &L, int prec);
hipError_t launch_gemv_t2(const WsLayout &L, void *ws, int prec, const double *a,
                          const double *b, const double *b_sub, const double *b_coef,
                          int *nblk, hipStream_t st);
// fixed-order reduction of the partials: ya/yb[c] = out_scale / (*out_div) * sum
hipError_t launch_t2_reduce(const WsLayout &L, void *ws, int nblk, double *ya, double *yb,
                            int64_t nout, double out_scale, const double *out_div, hipStream_t st);
hipError_t launch_energy_reduce(const WsLayout &L, void *ws, hipStream_t st);

// lanczos.hip
hipError_t launch_start_vector(double *v, int64_t L, int64_t ldv, int mode, uint64_t seed,
                               hipStream_t st);
// split: w = H~'v assembled as [g.v[1:]/2 ; g v0/2 + H_eff v[1:]] with g in FP64 (the
// operator pair then comes from an apply of (0, v[1:]))
hipError_t launch_lanczos_step(const WsLayout &L, void *ws, double *V, double *img, int j, int mode,
                               int split, uint64_t seed, hipStream_t st);
hipError_t launch_ritz(const WsLayout &L, void *ws, int m, int k, hipStream_t st);
hipError_t launch_restart_basis(const WsLayout &L, void *ws, const double *Vold, double *Vnew,
                                const double *Iold, double *Inew, int m, int k, int mode, uint64_t seed,
                                hipStream_t st);
hipError_t launch_ritz_vector(const WsLayout &L, void *ws, const double *V, const double *img, int m,
                              double *y, double *hy, hipStream_t st);
hipError_t launch_residual_image(const WsLayout &L, void *ws, const double *y, const double *hy, double *r,
                                 int mode, hipStream_t st);
hipError_t launch_connected_c0(const WsLayout &L, void *ws, const double *y, hipStream_t st);

// vmc.hip
int64_t vmc_scan_chunks(int64_t ns);
hipError_t launch_vmc_sample(const WsLayout &L, void *ws, const double *u, int64_t nsamp, int k, double Z,
                             int64_t *rows, double *out, hipStream_t st);
hipError_t launch_vmc_diag(const WsLayout &L, void *ws, double *w, double *u, int nb, hipStream_t st);
hipError_t launch_vmc_gather(const WsLayout &L, void *ws, const uint64_t *keys, int hfac, hipStream_t st);
hipError_t launch_vmc_diag_rows(const WsLayout &L, void *ws, int64_t nrows, double *w, double *u, hipStream_t st);
hipError_t launch_vmc_rhs_rows(const WsLayout &L, void *ws, int64_t nrows, double *y, hipStream_t st);
hipError_t launch_update(const WsLayout &L, void *ws, const double *y, double *dtheta,
                         double *theta, int64_t P, int mode, hipStream_t st);
hipError_t launch_copy(double *dst, const double *src, int64_t n, hipStream_t st);
hipError_t launch_reset_solve(const WsLayout &L, void *ws, hipStream_t st);

// grouped launches (batch): one work item per member for the vector kernels
enum GroupedOp {
    kGrpReset, kGrpStart, kGrpLanczos, kGrpRitz, kGrpRestart, kGrpRitzVector, kGrpResidual,
    kGrpUpdate, kGrpGather
};
// op-specific integer arguments: Start(mode, from_y), Lanczos(j, cur, mode, split),
// Ritz(m, k), Restart(cur, m, k, mode), RitzVector(cur, m), Residual(mode, split)
hipError_t launch_lanczos_grouped(int op, const Member *M, const WorkItem *items, int nitems,
                                  int i0, int i1, int i2, int i3, uint64_t seed,
                                  MemberScalars *out, hipStream_t st);
// row/tile work items: which = 0 apply (w -> u, [yS, yH] = D~^T [w, u]),
// which = 1 evaluation (psi -> H psi, gradient)
hipError_t launch_gemv_rows_grouped(const Member *M, const WorkItem *items, int nitems, int prec,
                                    int vsel, int j, int cur, int zero_v0, size_t lds_bytes,
                                    hipStream_t st);
hipError_t launch_gemv_t2_grouped(const Member *M, const WorkItem *items, int nitems, int prec,
                                  int which, hipStream_t st);
hipError_t launch_reduce_grouped(const Member *M, const WorkItem *items, int nitems, int which,
                                 hipStream_t st);
hipError_t launch_energy_grouped(const Member *M, const WorkItem *items, int nitems, int stage,
                                 hipStream_t st);
hipError_t launch_nqs_dtilde_grouped(const Member *M, const WorkItem *items, int nitems, int n,
                                     uint32_t flags, hipStream_t st);
constexpr int kGroupedT2Chunks = 8;   // chunks per lane of a grouped D~^T column tile

}  // namespace irl
