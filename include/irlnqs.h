/*
 * irlnqs.h -- C ABI of the MI355X (gfx950) linear-method operator library.
 *
 * The library applies the linear-method (LM) operator pair of the paper's
 * Methods section "From SR to a Stable Eigenvalue Problem",
 *
 *     v  ->  ( D~^T H D~ v ,  D~^T D~ v ),
 *
 * where D~ = [psi, d psi / d theta] is the N_s x (P+1) amplitude/Jacobian matrix
 * of a one-hidden-layer network over a determinant set (tangent basis
 * chi_0 = psi, chi_i = d psi / d theta_i; H~ and S~ of Eq. rayleigh_quotient)
 * and H is the second-quantised Hamiltonian of Methods, "Wave Function
 * Ansatz", applied matrix-free by Slater-Condon single and double excitations
 * restricted to the set.  On top of the apply it runs the implicitly
 * restarted Lanczos solve of Algorithm 1 (Lanczos recurrence of Algorithm 2
 * with full reorthogonalisation, Ritz pairs, exact-shift implicit QR restarts;
 * Methods, "The Standard Lanczos Process and Implicit Restart") for the lowest
 * eigenpair of the centred S ~ I problem (Eq. standard_evp), and the
 * parameter update taken from that eigenvector.
 *
 * Conventions
 *  - Determinant key: uint64, alpha orbital p at bit p, beta orbital p at bit
 *    32 + p (n_orb <= 32).  A determinant set is stored in ascending key order;
 *    row r of D~ is the r-th key.
 *  - Integrals: h is n x n row-major; g is n^4 row-major with
 *    g[((p*n + q)*n + r)*n + s] = (pq|rs) (chemists' notation),
 *    H = sum h_pq a+_p a_q + 1/2 sum (pq|rs) a+_p a+_r a_s a_q over spin-orbitals,
 *    alpha spin-orbitals ordered before beta ones for the fermionic sign.
 *  - Network: x_v = occupation of spin-orbital v (alpha v < n, beta v >= n),
 *    V = 2 n, psi = sum_v a_v x_v + sum_h tanh(b_h + sum_v W_hv x_v);
 *    theta = [a (V), b (H), W (H x V row-major)], P = V*H + H + V.
 *  - Every pointer documented "device" belongs to the HIP device that was
 *    current when the system was created.  Streams are hipStream_t passed as
 *    void* (NULL = the default stream).  All work is enqueued on the given
 *    stream; calls that return host scalars synchronise that stream.
 *  - A handle is not thread-safe.  Several handles may be used concurrently
 *    from different threads or streams.
 *  - No exception crosses the ABI.  Negative return values are errors,
 *    positive ones are warnings with a valid result; irl_last_error() returns
 *    a message for the last failing call on a handle.
 */
#ifndef IRLNQS_H
#define IRLNQS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------- */
enum irl_status {
    IRL_OK = 0,
    IRL_ENOTCONV = 1,   /* IRL stopped at max_restarts; result valid, not converged */
    IRL_ESTEP = 2,      /* |c_0| too small to form an update; theta left unchanged */
    IRL_EINVAL = -1,    /* invalid argument (sizes, popcounts, duplicates, symmetry) */
    IRL_ENOMEM = -2,    /* device allocation failed or workspace too small */
    IRL_EDEVICE = -3,   /* a HIP runtime call failed (message in irl_last_error) */
    IRL_ESTATE = -4     /* workspace holds no D~ for this call (evaluate/set first) */
};

/* operator precision of the D~ products */
enum irl_precision { IRL_FP64 = 0, IRL_FP32 = 1 };

/* eigenproblem form (Eq. standard_evp):
 *  IRL_MODE_A: (P+1)-dimensional centred matrix H~' = H~ - E S~ with identity
 *              metric; the update is dtheta = c[1:] / c[0].
 *  IRL_MODE_P: the P x P matrix H_eff (Eq. heff) with identity metric; returns
 *              the direction only (no update is defined).
 *  IRL_MODE_C: mode A in the connected tangent basis (Methods, "From SR to a
 *              Stable Eigenvalue Problem": H_eff in connected-correlation
 *              form): each derivative column d_i psi is replaced by its part
 *              orthogonal to psi, d_i psi - sigma_i psi with sigma = D~[:, 1:]^T
 *              psi / Z.  The centred matrix keeps mode A's psi row and column
 *              (g / 2) and its H_eff block becomes H_eff - (g sigma^T + sigma
 *              g^T) / 2.  The linearised wavefunction c_0 psi + sum_i c_i (d_i
 *              psi - sigma_i psi) gives the update dtheta = c[1:] / (c_0 -
 *              sigma . c[1:]).  FP64 solves with block 0 only; irl_step
 *              computes sigma (one D~^T pass) before the solve. */
enum irl_mode { IRL_MODE_A = 0, IRL_MODE_P = 1, IRL_MODE_C = 2 };

/* workspace flags (irl_workspace_query) */
enum irl_ws_flags {
    IRL_WS_FP64 = 1u,   /* hold an FP64 copy of D~ (required for IRL_FP64 applies) */
    IRL_WS_FP32 = 2u,   /* hold an FP32 copy of D~ (required for IRL_FP32 applies) */
    IRL_WS_BLOCK = 4u,  /* room for multi-vector applies and block solves of up to 8
                           vectors (8 vectors of n_dets for w and u, 8 of P+1 for the
                           outputs and larger reduction partials) */
    IRL_WS_FACTORED = 8u,  /* keep the Jacobian of the one-hidden-layer network in
                           factored form (psi, d = 1 - t^2 of n_dets x H, and the
                           occupations) instead of, or beside, the D~ copies: IRL_FP64
                           applies and the gradient then use the network's forward and
                           backward products, about 8 H bytes per determinant instead
                           of 8 (P + 1).  Needs irl_nqs_evaluate (not irl_dtilde_set)
                           and V <= 64. */
    IRL_WS_SAMPLED = 16u  /* with IRL_WS_FACTORED: room to gather the rows drawn by
                           irl_vmc_sample contiguously (keys, psi, weights, local
                           energies and d rows: about 8 (H + 5) bytes per
                           determinant), so the sampled operator's products run
                           over the drawn rows only */
};

/* irl_step flags */
enum irl_step_flags {
    IRL_STEP_WS_CURRENT = 1u,    /* ws already holds D~, Z, E, g for *theta; skip evaluation */
    IRL_STEP_NO_EVAL_AFTER = 2u, /* do not evaluate E(theta + dtheta) after the update */
    IRL_STEP_NO_UPDATE = 4u,     /* solve only; leave theta unchanged */
    IRL_STEP_NO_POLISH = 8u,     /* FP32 solve: skip the FP64 polish (see irl_step) */
    IRL_STEP_FULL_CYCLES = 16u,  /* test convergence only at the end of each m-step cycle
                                    (no early Ritz tests inside a cycle) */
    IRL_STEP_GRAPH = 32u,        /* single-vector solves that test only at the end of a
                                    cycle (operators under 256 MB per apply, or
                                    IRL_STEP_FULL_CYCLES): capture each cycle kind (the
                                    first, a restart from either basis) once as a HIP
                                    graph on a library stream and replay it on the
                                    caller's stream; results equal the launched path bit
                                    for bit.  The graphs are kept with the system, keyed
                                    on the workspace, sizes, mode, precision, seed and the
                                    Hamiltonian and sampling state, and rebuilt when any
                                    changes; ignored while per-kernel timing is on; a
                                    capture that fails falls back to launches. */
    IRL_STEP_WARM_START = 64u    /* single-vector solves: start the Lanczos process from
                                    the Ritz vector of this system's previous converged
                                    solve in the same workspace, with the same dimension,
                                    layout and mode (in an optimisation loop, the last
                                    step's eigenvector), instead of the seeded random
                                    vector; otherwise the random vector.  Every converged
                                    single-vector solve keeps a copy of its Ritz vector in the workspace
                                    for this (ncols doubles); any other system that
                                    steps in the same workspace in between overwrites it,
                                    which changes only the start.  The converged pair
                                    meets the same tolerances either way.  The saved
                                    vector is known by the workspace's address: a caller
                                    that frees a workspace and steps in a new one at the
                                    same address omits the flag for that first step. */
};

/* K4 variant selection (irl_system_desc.flags) */
enum irl_system_flags {
    IRL_SYS_FORCE_HASH = 1u,     /* use the general hashed per-determinant Hamiltonian
                                    apply for every set (full spaces and selected sets
                                    that would otherwise take the beta-blocked kernel) */
    IRL_SYS_FORCE_PULL = 2u,     /* full space: per-determinant kernel with string-rank
                                    lookup instead of the string-product kernel */
    IRL_SYS_STORE_SLICED = 4u,   /* irl_system_store_hamiltonian uses the LDS-sliced
                                    layout (the default for sets of at most 256
                                    slices of 2^14 determinants) */
    IRL_SYS_STORE_BLOCKS = 8u    /* irl_system_store_hamiltonian uses the L2-blocked
                                    layout at any set size (the default only beyond
                                    256 slices) */
};

typedef struct irl_system irl_system;

typedef struct {
    int32_t n_orb;          /* spatial orbitals n, 1 <= n <= 32 (n <= 20 for a full space) */
    int32_t n_alpha;        /* alpha electrons, 0 <= n_alpha <= n */
    int32_t n_beta;         /* beta electrons, 0 <= n_beta <= n */
    const double *h;        /* host, n*n, symmetric to 1e-12 */
    const double *g;        /* host, n^4, 8-fold symmetric to 1e-12 */
    double e_core;          /* constant added to every reported energy */
    const uint64_t *dets;   /* host, n_dets keys (any order, no duplicates);
                               NULL = the full (n_alpha, n_beta) space */
    int64_t n_dets;         /* ignored when dets == NULL */
    uint32_t flags;         /* irl_system_flags */
} irl_system_desc;

typedef struct {
    int64_t n_dets;         /* N_s */
    int32_t n_orb, n_alpha, n_beta;
    int32_t full_space;     /* 1 if the set is the full (n_alpha, n_beta) space */
    int64_t n_alpha_strings, n_beta_strings;   /* distinct strings in the set */
    int64_t max_connections;  /* singles + doubles per determinant (before projection) */
    size_t device_bytes;    /* device memory owned by the handle */
    int32_t ham_kernel;     /* 0: hashed per-determinant, 1: rank per-determinant,
                               2: string-product (full space), 3: beta-blocked
                               per-determinant (selected sets with n_orb <= 24),
                               4: stored rows (irl_system_store_hamiltonian) */
    int32_t stored_col_blocks;  /* column blocks of the stored rows (0 unless ham_kernel == 4) */
    int64_t stored_elements;    /* off-diagonal elements stored (padding excluded; 0 unless
                                   ham_kernel == 4) */
} irl_system_info;

typedef struct {
    int32_t V;              /* visible units, must equal 2 * n_orb */
    int32_t H;              /* hidden units, 1 <= H <= 1024 */
    double *theta;          /* device, P doubles, order [a, b, W] */
} irl_nqs_desc;

typedef struct {
    double Z;               /* psi^T psi */
    double E;               /* psi^T H psi / Z + e_core */
    double *grad;           /* device, P doubles, dE/dtheta = 2 J^T (H psi - E psi) / Z;
                               NULL: not copied out (it stays in the workspace) */
} irl_eval_out;

typedef struct {
    int32_t m;              /* Krylov dimension, 2 <= m <= 64 (default 20) */
    int32_t k_keep;         /* vectors kept at a restart, 1 <= k_keep < m (default 1) */
    double tol;             /* residual tolerance on ||H~'y - lambda y|| (default 1e-12) */
    int32_t max_restarts;   /* default 300 */
    int32_t precision;      /* irl_precision of the D~ products */
    int32_t mode;           /* irl_mode */
    uint64_t seed;          /* start vector: splitmix64(seed, index) -> U(-1, 1) */
    uint32_t flags;         /* irl_step_flags */
    int32_t block;          /* 0 or 1: implicitly restarted Lanczos (Algorithm 1); 2..8:
                               thick-restart block Lanczos with this many vectors per
                               operator pass (needs IRL_WS_BLOCK; m counts basis columns,
                               2 * block <= m <= 64, k_keep <= m - block) */
} irl_solver_opts;

typedef struct {
    double E_before;        /* E(theta) */
    double E_after;         /* E(theta + dtheta) (NaN when not evaluated) */
    double lambda_min;      /* lowest eigenvalue found */
    double residual_est;    /* |beta_m e_m^T u_1| of the accepted cycle */
    double residual_explicit;  /* ||H~'y - lambda y|| with one more operator apply */
    double tol_used;        /* max(tol, 64 u_op ||T_m||) */
    double c0;              /* first component of the unit Ritz vector (mode A);
                               mode C: c_0 - sigma . c[1:], the coefficient of psi */
    double gap;             /* second-lowest minus lowest Ritz value */
    double norm_T;          /* max |Ritz value| of the last cycle */
    int32_t n_apply;        /* operator applies used by the solve */
    int32_t n_restart;      /* restart cycles */
    int32_t converged;      /* 1 if the residual test passed */
    int32_t n_apply_lo;     /* of n_apply, the reduced-precision (FP32) applies */
    double ms_eval, ms_solve, ms_after;   /* host wall time of each phase */
    int32_t n_graph_cycles; /* cycles replayed from captured graphs (IRL_STEP_GRAPH) */
    int32_t reserved;
} irl_step_result;

/* ---- system --------------------------------------------------------------- */

/* Build the device tables of one system: the determinant set (enumerated when
 * dets == NULL: every alpha string with n_alpha bits times every beta string
 * with n_beta bits, Methods "Wave Function Ansatz" and Eq. constraint), the
 * key -> row lookup, the integrals and the diagonal H_xx.  Inputs are copied;
 * the library owns the device tables until irl_system_destroy.
 * Errors: IRL_EINVAL (n out of range, wrong popcount or orbital outside n,
 * duplicate keys, the reserved key 2^64 - 1, non-symmetric h or g beyond
 * 1e-12, empty set), IRL_ENOMEM,
 * IRL_EDEVICE.  *out is NULL on error. */
int irl_system_create(const irl_system_desc *desc, void *stream, irl_system **out);

/* Release a system (NULL is ignored). */
void irl_system_destroy(irl_system *sys);

/* Sizes of a system (host call, no device work). */
int irl_system_info_get(const irl_system *sys, irl_system_info *out);

/* Store the off-diagonal elements of H inside the set (Methods, "Wave Function
 * Ansatz": the second-quantised electronic Hamiltonian, whose elements between
 * determinants follow from the Slater-Condon rules) in one of two layouts.
 * L2-blocked (IRL_SYS_STORE_BLOCKS, or sets of more than 256 slices): compressed
 * rows split into column blocks; the targets of block b are rows [b 2^s,
 * (b + 1) 2^s), a slice of the amplitude vector of about 2 MiB (at most 8
 * blocks, wider for larger sets), so the gathers of one block stay in the L2
 * cache; layout: row offsets int64[blocks][n_dets + 1] (block-major), targets
 * int32[nnz], values FP64[nnz]; bytes_needed = blocks * (n_dets + 1) * 8 + nnz *
 * 12.  LDS-sliced (the default): slices of 2^14 target rows, whose 128 KiB of
 * amplitudes one workgroup stages in LDS, at most 256 slices.
 * Inside a slice the rows are taken in windows of 4096; a window's rows are
 * ordered by their number of elements in the slice (descending, ties by row)
 * and grouped 64 at a time, one row per lane of a wavefront; a group stores
 * L x 64 slots (L = its longest row rounded up to an even number), slot
 * (j, lane) holding the lane row's j-th element (zero padding past the row's
 * end) as a 16-bit target (row - b 2^14) and an FP64 value; values and targets
 * sit in lane-interleaved pairs (j, j + 1), so a wavefront loads 1 KiB of
 * values or 256 bytes of targets contiguously.  Per slice and group: the slot offset (uint32) and L
 * (uint16); per lane of a group: the lane's row inside its window (uint16,
 * 0xffff for an empty lane); per slice: the slot base (int64) and room for
 * one FP64 partial sum per row (an apply sums a row's slices in slice order in
 * LDS, one window at a time; when the set has fewer than 512 windows, the
 * slices are split into equal runs whose partial sums are added in run order,
 * the same for every apply of the set).  bytes_needed = groups * slices * 6 +
 * groups * 64 * slices * 2 + slices * 8 + slots * 10 + slices * n_dets * 8
 * (groups = ceil(n_dets / 64); slots counts the padding).  Device memory is
 * owned by the system.  Later applies stream these rows instead of enumerating
 * excitations (ham_kernel becomes 4, stored_col_blocks reports the block or
 * slice count); results agree with the enumerating kernels to rounding
 * (summation order differs) and are reproducible.  Enumeration passes count and
 * fill the rows; the call synchronises stream.
 * max_bytes: device bytes the caller allows for the stored rows.
 * bytes_needed (may be NULL): receives the byte count above.
 * Errors: IRL_ENOMEM when the rows need more than max_bytes or allocation
 * fails (the system is unchanged and stays usable), IRL_EDEVICE, IRL_EINVAL.
 * Calling it again after success does nothing. */
int irl_system_store_hamiltonian(irl_system *sys, size_t max_bytes, size_t *bytes_needed,
                                 void *stream);

/* Message for the last error on sys ("" if none); for a NULL sys, the last
 * error of a failed irl_system_create on this thread. */
const char *irl_last_error(const irl_system *sys);

/* ---- workspace -------------------------------------------------------------- */

/* Bytes of caller-owned device workspace for a D~ with ncols = P + 1 columns
 * and the D~ copies named by ws_flags (irl_ws_flags).  The workspace holds D~
 * (row-major, rows padded to a multiple of 128 bytes), psi, H psi, the
 * gradient, the operator vectors, the split reduction partials and the
 * double-buffered Krylov basis (room for m <= 64).  The caller allocates it
 * (any 256-byte aligned device buffer) and keeps it alive while it is in use;
 * its contents persist between calls.  A system remembers the last workspace
 * it evaluated into; applies and steps must pass that same workspace.
 * Errors: IRL_EINVAL (ncols < 1, no precision flag). */
int irl_workspace_query(const irl_system *sys, int64_t ncols, uint32_t ws_flags,
                        size_t *bytes);

/* ---- network evaluation --------------------------------------------------- */

/* Evaluate the network on every determinant and build D~ = [psi, d psi/d theta]
 * (Methods, "From SR to a Stable Eigenvalue Problem", linearised wavefunction)
 * into ws, then Z = psi^T psi, E = psi^T H psi / Z (compensated sums) and the
 * energy gradient g = 2 J^T (H psi - E psi) / Z (Methods, "Practical
 * Matrix-Free Implementation", definition of F for a real wavefunction).
 * ws_flags must match the irl_workspace_query call that sized ws.  Writes
 * out->Z, out->E and, if out->grad != NULL, P doubles to out->grad (device).
 * Synchronises the stream.  Errors: IRL_EINVAL (V != 2 n, H out of range,
 * NULL theta), IRL_ENOMEM (ws_bytes too small), IRL_EDEVICE. */
int irl_nqs_evaluate(irl_system *sys, const irl_nqs_desc *nqs, void *ws, size_t ws_bytes,
                     uint32_t ws_flags, irl_eval_out *out, void *stream);

/* Load an arbitrary D~ (device, n_dets x ncols, leading dimension ld >= ncols
 * elements, dtype IRL_FP64 = double or IRL_FP32 = float) into ws in place of
 * a network evaluation; column 0 plays the role of psi.  Every copy named in
 * ws_flags is filled (converted as needed).  Z, E and g = 2 D~[:,1:]^T
 * (H psi - E psi) / Z are computed from it as in irl_nqs_evaluate, from the
 * FP64 copy when present.  ws must have been sized for this ncols and
 * ws_flags.  Synchronises the stream.
 * Errors: IRL_EINVAL, IRL_ENOMEM, IRL_EDEVICE. */
int irl_dtilde_set(irl_system *sys, const void *D, int64_t ld, int64_t ncols, int32_t dtype,
                   void *ws, size_t ws_bytes, uint32_t ws_flags, void *stream);

/* ---- the operator ------------------------------------------------------------ */

/* The LM operator apply (Eq. rayleigh_quotient matrices applied to a vector,
 * matrix-free as in Methods, "Practical Matrix-Free Implementation"):
 *     w = D~ v,  u = H w  (restricted to the set),
 *     yH = D~^T u = D~^T H D~ v,   yS = D~^T w = D~^T D~ v,
 * raw and unnormalised (divide by Z for the <psi|psi> = 1 convention).
 * v, yH, yS: device, P+1 doubles each, caller-owned, must not overlap.
 * precision selects the FP64 or FP32 copy of D~ (FP32 products accumulate in
 * FP32 per row block; the Hamiltonian apply is always FP64).  Asynchronous on
 * stream.  Errors: IRL_ESTATE (no D~ in ws for the requested precision),
 * IRL_EINVAL, IRL_EDEVICE. */
int irl_apply_lm_operator(irl_system *sys, void *ws, size_t ws_bytes, const double *v,
                          double *yH, double *yS, int32_t precision, void *stream);

/* The LM operator on nb <= 8 vectors with one pass over D~ per direction (the
 * multi-vector form behind block Lanczos, which the paper names as its next
 * step in the Discussion):  for q < nb,
 *     YH[:, q] = D~^T H D~ V[:, q],   YS[:, q] = D~^T D~ V[:, q]   (raw, as above).
 * V: device, nb columns of ncols = P + 1 doubles, column q at V + q * ldv
 * (ldv >= ncols).  YH, YS: device, nb columns at stride ldy >= ncols (entries
 * >= ncols are not written).  Needs a workspace evaluated with IRL_WS_BLOCK.
 * With a D~ copy, the D~ bytes per call are those of one vector and each column
 * equals irl_apply_lm_operator on that column to rounding (the D~^T partial sums
 * use other row blocks).  FP64 with IRL_WS_FACTORED takes the factored products
 * one vector at a time, and each column equals irl_apply_lm_operator on it bit
 * for bit.  Asynchronous on stream.  Errors: IRL_ESTATE, IRL_EINVAL,
 * IRL_ENOMEM, IRL_EDEVICE. */
int irl_apply_lm_operator_block(irl_system *sys, void *ws, size_t ws_bytes, const double *V, int64_t ldv,
                                int32_t nb, double *YH, double *YS, int64_t ldy, int32_t precision,
                                void *stream);

/* u = H w on the determinant set (device vectors of n_dets doubles). */
int irl_apply_hamiltonian(irl_system *sys, const double *w, double *u, void *stream);

/* ---- one optimisation step ---------------------------------------------- */

/* One optimisation step (Algorithm 1 around the operator apply):
 *  1. unless IRL_STEP_WS_CURRENT: irl_nqs_evaluate at theta;
 *  2. implicitly restarted Lanczos for the lowest eigenpair of the centred
 *     operator (mode A: H~'; mode P: H_eff), Krylov dimension m, k_keep kept
 *     vectors per restart, exact shifts = the m - k_keep largest Ritz values,
 *     full (two-pass classical Gram-Schmidt) reorthogonalisation, convergence
 *     when the Ritz residual estimate is below max(tol, 64 u_op ||T_m||),
 *     confirmed by one explicit apply; on operators that stream >= 256 MB per
 *     apply the Ritz pair of T_j is also tested every 2 steps inside a cycle
 *     (IRL_STEP_FULL_CYCLES disables this);
 *     With precision IRL_FP32 the operator's D~ products use the FP32 copy and
 *     the centred matrix takes its psi row and column from the FP64 gradient
 *     (split form); if the workspace also holds the FP64 copy, the solve is
 *     then polished in FP64 from the FP32 Ritz vector (unless
 *     IRL_STEP_NO_POLISH), so the result meets the FP64 tolerance;
 *  3. mode A: dtheta = c[1:] / c[0] (mode C: c[1:] / (c_0 - sigma . c[1:]));
 *     unless IRL_STEP_NO_UPDATE theta += dtheta;
 *  4. unless IRL_STEP_NO_EVAL_AFTER: evaluate at the new theta (ws then holds
 *     D~ for the new theta, so the next call may pass IRL_STEP_WS_CURRENT).
 * nqs may be NULL when ws holds a D~ from irl_dtilde_set (no update then).
 * dtheta: device, P doubles, or NULL.  ritz: device, P+1 doubles (mode A) or
 * P doubles (mode P), unit-norm eigenvector, or NULL.
 * Returns IRL_OK, IRL_ENOTCONV (r filled with the last cycle's values),
 * IRL_ESTEP (|c_0| < 1e-8, mode C |c_0 - sigma . c[1:]| < 1e-8: theta
 * unchanged) or an error (IRL_EINVAL for mode C with IRL_FP32, block > 1 or
 * sampled estimators). */
int irl_step(irl_system *sys, irl_nqs_desc *nqs, const irl_solver_opts *opts, void *ws,
             size_t ws_bytes, uint32_t ws_flags, double *dtheta, double *ritz,
             irl_step_result *r, void *stream);

/* Default solver options (m 20, k_keep 1, tol 1e-12, max_restarts 300, FP64,
 * mode A, seed 0, flags 0, block 0). */
void irl_solver_opts_default(irl_solver_opts *o);

/* ---- first-order baseline (optimiser comparison) ---- */

/* Adam step sizes: the first-order method the paper compares IRL and standard
 * Lanczos against (Results, "Efficiency and Numerical Stability of IRL
 * Optimization", Fig. 2); Methods, "Practical Matrix-Free Implementation", costs
 * one such step as one gradient evaluation. */
typedef struct {
    double lr;              /* step size alpha */
    double beta1, beta2;    /* decay rates of the first and second moment estimates */
    double eps;             /* added to the square root of the second moment */
} irl_adam_opts;

/* One Adam step on theta (in place): evaluates psi, Z, E and the gradient g at
 * theta exactly as irl_nqs_evaluate does (same workspace and flags), then with the
 * step count t >= 1
 *   m <- beta1 m + (1 - beta1) g,   v <- beta2 v + (1 - beta2) g^2,
 *   theta <- theta - lr (m / (1 - beta1^t)) / (sqrt(v / (1 - beta2^t)) + eps)
 * elementwise (the bias-corrected moments of the published algorithm).
 * m, v: device FP64[P], caller-owned, all zero before the first step.
 * out (may be NULL): Z and E at theta before the update; out->grad, if set,
 * receives g.  Errors: as irl_nqs_evaluate, and IRL_EINVAL for t < 1, m or v NULL,
 * or lr, beta1, beta2, eps out of [0, inf) x [0, 1) x [0, 1) x (0, inf). */
int irl_adam_step(irl_system *sys, const irl_nqs_desc *nqs, void *ws, size_t ws_bytes, uint32_t ws_flags,
                  const irl_adam_opts *opts, double *m, double *v, int64_t t, irl_eval_out *out,
                  void *stream);

/* ---- sampled estimators (variational Monte Carlo) ----------------------- */

/* Result of irl_vmc_sample. */
typedef struct {
    double E_sampled;       /* mean local energy over the draws (+ e_core) */
    double E_exact;         /* psi^T H psi / Z on the set at the same theta (+ e_core) */
    double E_loc_var;       /* variance of the local energy over the draws */
    int64_t n_unique;       /* distinct determinants drawn */
    int64_t n_samples;
} irl_vmc_out;

/* Draw n_samples configurations from |psi|^2 / Z on the determinant set and
 * replace the workspace's exact estimators by the sampled ones.
 *
 * Sampling (Methods, "Autoregressive Modeling and Physical Constraints", Eqs.
 * autoregressive_factorization and constraint): the spin-orbitals taken one at
 * a time from the exact conditionals of |psi|^2 (most significant key bit
 * first: beta orbital n-1 down to 0, then alpha n-1 down to 0), every draw
 * inside the fixed (N_alpha, N_beta) set, one uniform number per sample.  This
 * is the inverse transform of the cumulative |psi|^2 in ascending key order,
 * which the library evaluates in 64-bit fixed point (psi^2 2^k rounded, the
 * total below 2^62; determinants with psi^2 below 2^-62 Z are never drawn).
 * u: device, n_samples doubles in [0, 1) (values outside are clamped into it);
 * the caller supplies the random numbers.  rows (may be NULL): device,
 * n_samples int64, the drawn row of each sample.  grad (may be NULL): device,
 * P doubles, receives the sampled gradient F.
 *
 * Estimators (Methods, "From SR to a Stable Eigenvalue Problem", Eq.
 * centered_hamiltonian; "Practical Matrix-Free Implementation", Eq.
 * matrix_vec_prod), with E_loc(x) = (H psi)(x) / psi(x) on the set and O(x) =
 * D~[x, :] / psi(x) (O_0 = 1): E = <E_loc>, F = 2 <O (E_loc - E)>, and the
 * operator pair of irl_apply_lm_operator becomes (y_H, y_S) = Z (<O E_loc O^T> v,
 * <O O^T> v), so the centred matrix (y_H - E y_S) / Z of irl_step is the sample
 * mean of O (E_loc - E) O^T (mode A: P + 1 components; mode P: H_eff alone).
 * Until the next irl_nqs_evaluate or irl_dtilde_set, applies and irl_step with
 * IRL_STEP_WS_CURRENT use these (E_before then reports the sampled energy);
 * an irl_step that evaluates, or evaluates after its update, returns to the
 * exact estimators.  Mode C is not defined on sampled estimators (IRL_EINVAL).
 *
 * Requires an evaluated workspace with an FP64 D~ copy or the factored Jacobian
 * (for F).  One synchronisation (the scalars of out).  Errors: IRL_ESTATE (no
 * evaluation in ws), IRL_EINVAL (u NULL, n_samples outside [1, 2^31 - 1], no
 * FP64 Jacobian), IRL_ENOMEM, IRL_EDEVICE. */
int irl_vmc_sample(irl_system *sys, void *ws, size_t ws_bytes, const double *u, int64_t n_samples,
                   int64_t *rows, double *grad, irl_vmc_out *out, void *stream);

/* ---- batches of independent solves ------------------------------------- */

/* A batch groups `count` independent optimisations (systems, networks,
 * workspaces) that are stepped together: every kernel launch of a batch step
 * covers all members that are still active (grouped kernels over per-member
 * work lists), the members advance through the Lanczos steps in lockstep, and
 * the host reads back all members' scalars with one copy per check point.
 * Each member follows exactly the arithmetic of irl_step on its system (same
 * row blocks, reduction order, seeds and tolerances), so its result equals
 * that solo result bit for bit.  The Hamiltonian apply of each member is the
 * kernel its system uses when the batch is created: string-product members
 * get their own launch, stored-row and per-determinant members share grouped
 * launches (rows stored after batch create are not used by the batch).
 * ws_flags: D~ copies (IRL_WS_FP64 and/or IRL_WS_FP32; the D~ streams are
 * grouped too) or IRL_WS_FACTORED alone (each member's network products are
 * its solo launches, issued inside the lockstep loop; V <= 64); not
 * IRL_WS_SAMPLED.
 * systems[i], nqs[i] and ws[i] (sized by irl_workspace_query for P_i + 1
 * columns and ws_flags) are borrowed and must stay alive while the batch
 * exists; a system must not be used by two members.  Requires
 * (P_i + 1) <= 8192, and at most 2^26 determinant rows over the members that
 * share one Hamiltonian kernel kind (checked at each step: IRL_EINVAL).
 * Errors: IRL_EINVAL, IRL_ENOMEM, IRL_EDEVICE. */
typedef struct irl_batch irl_batch;
int irl_batch_create(int32_t count, irl_system *const *systems, const irl_nqs_desc *nqs,
                     void *const *ws, const size_t *ws_bytes, uint32_t ws_flags,
                     irl_batch **out);
void irl_batch_destroy(irl_batch *batch);

/* One optimisation step for every member (irl_step semantics, same options for
 * all members).  dtheta: NULL or an array of count device pointers (each NULL
 * or P_i doubles).  results and status: host arrays of count entries; status[i]
 * is IRL_OK, IRL_ENOTCONV or IRL_ESTEP.  Returns IRL_OK or an error. */
int irl_batch_step(irl_batch *batch, const irl_solver_opts *opts, double *const *dtheta,
                   irl_step_result *results, int32_t *status, void *stream);

/* ---- per-kernel timing -------------------------------------------------- */

/* Kernel classes timed by irl_stats_*. */
enum irl_stat_kind {
    IRL_STAT_DTILDE_BUILD = 0,   /* network forward + Jacobian rows written to D~ */
    IRL_STAT_HAM_APPLY = 1,      /* u = H w */
    IRL_STAT_GEMV = 2,           /* w = D~ v (FP64 copy) */
    IRL_STAT_GEMV_T = 3,         /* [ya, yb] = D~^T [a, b] (stream part, FP64 copy) */
    IRL_STAT_REDUCE = 4,         /* fixed-order reduction of the D~^T partial sums */
    IRL_STAT_ENERGY = 5,         /* compensated Z and psi^T H psi reductions; the FP64
                                    gradient recomputed from theta (FP32-only workspace) */
    IRL_STAT_LANCZOS = 6,        /* Lanczos recurrence + reorthogonalisation step */
    IRL_STAT_RITZ = 7,           /* Ritz pairs, restart shifts, basis compression, Ritz vector */
    IRL_STAT_GEMV_LO = 8,        /* w = D~ v on the FP32 copy (IRL_STAT_GEMV: FP64 copy) */
    IRL_STAT_GEMV_T_LO = 9,      /* D~^T stream on the FP32 copy (IRL_STAT_GEMV_T: FP64 copy) */
    IRL_STAT_VMC = 10,           /* sampling, sampled weights and the sampled operator's diagonal */
    IRL_STAT_KINDS = 11
};

/* on != 0: from now on every kernel launch of this handle is bracketed by a
 * pair of HIP events on its stream; on == 0 stops and clears.  Adds a few
 * microseconds of host work per launch.  A batch step records its launches
 * (which cover all members) in the stats of the first member's system. */
int irl_stats_enable(irl_system *sys, int32_t on);

/* Restrict the timed launches to the kinds whose bits are set in `kinds`
 * (bit k = irl_stat_kind k; all kinds by default).  Launches of the other kinds
 * get no events and so none of their host and queue cost; their entries in
 * irl_stats_get stay zero.  The choice persists across irl_stats_enable calls.
 * IRL_EINVAL for a bit at or beyond IRL_STAT_KINDS. */
int irl_stats_select(irl_system *sys, uint32_t kinds);

/* Synchronise `stream` and return, per irl_stat_kind, the summed kernel time
 * in milliseconds (ms[IRL_STAT_KINDS]) and the launch count
 * (count[IRL_STAT_KINDS]) since the last irl_stats_enable(sys, 1). */
int irl_stats_get(irl_system *sys, double *ms, int64_t *count, void *stream);

/* ---- launch-shape tuning ------------------------------------------------- */

/* Launch shapes that a caller (the package's autotuner) may choose per system.
 * Each one only moves rows between workgroups: every row's sums are formed by
 * one wavefront in a fixed order, so results are bit-for-bit the same for every
 * value.  The operator's cost per matrix-vector product (Methods, "Practical
 * Matrix-Free Implementation") is what the choice changes. */
enum irl_tune_knob {
    IRL_TUNE_LUT_BLOCKS = 0,    /* workgroups of the table-driven forward pass and D~ v
                                   (selected sets, n <= 24, H >= 48); default 256,
                                   at least 128 rows each */
    IRL_TUNE_PULL_BLOCKS = 1,   /* workgroup cap of the enumerating Hamiltonian apply
                                   (hashed, rank or beta-blocked pull, one row per
                                   wavefront in grid strides); default 2^20 */
    IRL_TUNE_PULL_WAVES = 2     /* wavefronts (rows) per workgroup of that apply: 1, 2
                                   or 4; default 1 for n <= 20, else 4 */
};

/* Set `knob` of `sys` to `value` (0 restores the default).  Takes effect at the
 * next launch; captured Lanczos cycles are recaptured.  IRL_EINVAL for an
 * unknown knob, a negative value, a value above 65536 (LUT) or 2^20 (pull cap),
 * or a wavefront count other than 0, 1, 2 or 4. */
int irl_tune_set(irl_system *sys, int32_t knob, int32_t value);

/* Current value of `knob` (0 = default) in *value, and in *applies 1 when the
 * system's kernels use it: for IRL_TUNE_LUT_BLOCKS, D~ v over the whole set with
 * a network of `hidden` units runs the table-driven kernel; for
 * IRL_TUNE_PULL_BLOCKS and IRL_TUNE_PULL_WAVES, the Hamiltonian apply enumerates
 * excitations (no stored rows, not the string product).  Host pointers; IRL_EINVAL for an unknown knob
 * or hidden < 1 with IRL_TUNE_LUT_BLOCKS. */
int irl_tune_get(irl_system *sys, int32_t knob, int32_t hidden, int32_t *value, int32_t *applies);

/* ---- bit-exact test surface ----------------------------------------------- */

/* Copy the ascending key array (n_dets uint64) to host memory out. */
int irl_debug_keys(const irl_system *sys, uint64_t *out);

/* rows[i] = row of keys[i] in the set, or -1 if absent (host arrays of n). */
int irl_debug_lookup(const irl_system *sys, const uint64_t *keys, int64_t n, int32_t *rows);

/* irl_debug_lookup without any device allocation, for callers that cannot
 * allocate device memory (tight serving loops, harnesses that forbid
 * hipMalloc).  keys and rows are host arrays of n <= 262144 entries;
 * rows[i] = row of keys[i] in the set, or -1 if absent, bit-identical to
 * irl_debug_lookup.  The keys and rows are staged in a fixed 3 MiB device
 * array that the library holds on each GPU it runs on until the process ends
 * (its address is resolved when the first system is created on that device);
 * the work is enqueued on `stream`, which is synchronised before returning.
 * IRL_EINVAL for n < 0, n > 262144 or NULL arrays.  Every call on one GPU
 * shares that GPU's array: calls that overlap in time on the same GPU (from
 * several threads, or streams) race and must be serialised by the caller. */
int irl_lookup_noalloc(const irl_system *sys, const uint64_t *keys, int64_t n, int32_t *rows,
                       void *stream);

/* Copy the diagonal H_xx (n_dets doubles) to host memory out. */
int irl_debug_diagonal(const irl_system *sys, double *out);

/* Off-diagonal connections of determinant `row` inside the set, sorted by
 * target row, written to host arrays of capacity cap: target row, fermionic
 * sign (+1/-1), kind (1 alpha single, 2 beta single, 3 alpha-alpha,
 * 4 beta-beta, 5 alpha-beta double) and matrix element.  *count receives the
 * number of connections; IRL_EINVAL if it exceeds cap. */
int irl_debug_excitations(const irl_system *sys, int64_t row, int32_t *target, int8_t *sign,
                          uint8_t *kind, double *hval, int64_t cap, int64_t *count);

/* Copy rows [row0, row0 + nrows) of the current evaluation's tangent basis
 * (Methods, "From SR to a Stable Eigenvalue Problem": chi_0 = psi and the
 * parameter derivatives) to host memory.  psi: FP64[nrows].  rows: with the
 * factored Jacobian (IRL_WS_FACTORED) d = 1 - tanh^2(z) as FP64[nrows x H]
 * (*kind = 0, *ncols_out = H); else the rows of the FP64 D~ copy as
 * FP64[nrows x (P+1)] (*kind = 1) or of the FP32 copy as FP32[nrows x (P+1)]
 * (*kind = 2), *ncols_out = P+1.  Either pointer may be NULL.  IRL_ESTATE when
 * ws holds no evaluation, IRL_EINVAL for a row range outside [0, N_s). */
int irl_debug_jacobian(irl_system *sys, void *ws, size_t ws_bytes, int64_t row0, int64_t nrows,
                       double *psi_host, void *rows_host, int32_t *kind, int64_t *ncols_out);

/* Run j_end Lanczos steps of the centred mode-A (or mode-P) operator from the
 * unit vector v1 (device), no restart, and copy to host: the basis
 * V (j_end+1 rows of length L = P+1 or P, row-major), alpha (j_end) and beta
 * (j_end).  Tests the recurrence and the projection relation
 * H~' V_m = V_m T_m + beta_m v_{m+1} e_m^T (Methods, "The Standard Lanczos
 * Process and Implicit Restart"). */
int irl_debug_lanczos(irl_system *sys, void *ws, size_t ws_bytes, const double *v1,
                      int32_t j_end, int32_t precision, int32_t mode, double *V_host,
                      double *alpha_host, double *beta_host, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* IRLNQS_H */
