// C ABI of the LM-operator library: system set-up, network evaluation, the
// operator apply and the implicitly restarted Lanczos optimisation step.
// Host orchestration only; every arithmetic step runs in the HIP kernels of
// system.hip, hamiltonian.hip, nqs.hip, dtilde.hip and lanczos.hip.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <limits>
#include <string>
#include <vector>

#include "internal.h"

using namespace irl;

namespace {

thread_local std::string g_create_err;

int set_err(irl_system *s, int code, const std::string &msg)
{
    if (s)
        s->err = msg;
    else
        g_create_err = msg;
    return code;
}

#define CK(s, call)                                                                          \
    do {                                                                                     \
        hipError_t e_ = (call);                                                              \
        if (e_ != hipSuccess)                                                                \
            return set_err((s), IRL_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

int64_t binom_host(int n, int k)
{
    if (k < 0 || k > n) return 0;
    int64_t r = 1;
    for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
    return r;
}

double now_ms()
{
    using namespace std::chrono;
    return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

template <typename T>
int dev_alloc(irl_system *s, T **p, size_t count)
{
    size_t bytes = count * sizeof(T);
    if (bytes == 0) bytes = sizeof(T);
    hipError_t e = hipMalloc((void **)p, bytes);
    if (e != hipSuccess) {
        *p = nullptr;
        return set_err(s, IRL_ENOMEM, std::string("hipMalloc failed: ") + hipGetErrorString(e));
    }
    s->dev_bytes += bytes;
    return IRL_OK;
}

void free_cycle_graphs(irl_system *s);

void free_system(irl_system *s)
{
    if (!s) return;
    free_cycle_graphs(s);
    if (s->capture_stream) (void)hipStreamDestroy(s->capture_stream);
    free_dense_doubles(s);
    void *ptrs[] = {s->d.keys, s->d.h, s->d.g, s->d.diag, s->d.hkeys, s->d.hrows, s->d.rankA,
                    s->d.rankB, s->d.strA, s->d.strB, s->d.sglA, s->d.sglB, s->d.fA, s->d.fB,
                    s->d.dblA_rank, s->d.dblA_val, s->d.dblB_rank, s->d.dblB_val, s->d.jA,
                    s->d.jB, s->d.sglA_ia, s->d.sglB_ia, s->d.hfilter, s->d.bidx, s->d.bstart,
                    s->d.aidx, s->d.astart, s->d.arow, s->d.abeta,
                    s->d.hptr, s->d.hcol, s->d.hval, s->d.sbase, s->d.sgbase, s->d.sglen, s->d.sperm,
                    s->d.scol, s->d.sval, s->d.spart};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    if (s->host_scal) (void)hipHostFree(s->host_scal);
    for (hipEvent_t e : s->ev_pool) (void)hipEventDestroy(e);
    delete s;
}

int stats_fold(irl_system *s);

// read the scalar header of a workspace (synchronises the stream)
int read_scalars(irl_system *s, void *ws, const WsLayout &L, hipStream_t st)
{
    const size_t n = offsetof(WsScalars, alpha) + 4 * kMaxKrylov * sizeof(double);
    CK(s, hipMemcpyAsync(s->host_scal, ws_ptr<char>(ws, L.off_scal), n, hipMemcpyDeviceToHost, st));
    CK(s, hipStreamSynchronize(st));
    return stats_fold(s);
}

int check_ws(irl_system *s, void *ws, size_t ws_bytes, const WsLayout &L)
{
    if (!ws) return set_err(s, IRL_EINVAL, "workspace is NULL");
    if (reinterpret_cast<uintptr_t>(ws) % 256 != 0)
        return set_err(s, IRL_EINVAL, "workspace must be 256-byte aligned");
    if (ws_bytes < L.total)
        return set_err(s, IRL_ENOMEM, "workspace too small: need " + std::to_string(L.total) +
                                          " bytes, got " + std::to_string(ws_bytes));
    return IRL_OK;
}

// ---- per-kernel timing: event pairs around launches, folded after syncs ----
int stats_fold(irl_system *s)
{
    for (size_t i = 0; i < s->ev_used; ++i) {
        float ms = 0.f;
        CK(s, hipEventSynchronize(s->ev_pool[2 * i + 1]));
        CK(s, hipEventElapsedTime(&ms, s->ev_pool[2 * i], s->ev_pool[2 * i + 1]));
        s->stat_ms[s->ev_kind[i]] += ms;
        s->stat_cnt[s->ev_kind[i]] += 1;
    }
    s->ev_used = 0;
    return IRL_OK;
}

int stat_begin(irl_system *s, int kind, hipStream_t st)
{
    s->ev_open = false;
    if (!s->stats_on || !((s->stat_mask >> kind) & 1u)) return IRL_OK;
    const size_t cap = 4096;
    if (s->ev_used == cap) {
        int rc = stats_fold(s);
        if (rc) return rc;
    }
    while (s->ev_pool.size() < 2 * (s->ev_used + 1)) {
        hipEvent_t e;
        CK(s, hipEventCreate(&e));
        s->ev_pool.push_back(e);
    }
    if (s->ev_kind.size() < s->ev_used + 1) s->ev_kind.resize(s->ev_used + 1);
    s->ev_kind[s->ev_used] = kind;
    CK(s, hipEventRecord(s->ev_pool[2 * s->ev_used], st));
    s->ev_open = true;
    return IRL_OK;
}

int stat_end(irl_system *s, hipStream_t st)
{
    if (!s->stats_on || !s->ev_open) return IRL_OK;
    s->ev_open = false;
    CK(s, hipEventRecord(s->ev_pool[2 * s->ev_used + 1], st));
    s->ev_used += 1;
    return IRL_OK;
}

#define TIMED(s, kind, st, call)                       \
    do {                                               \
        int rc_ = stat_begin((s), (kind), (st));       \
        if (rc_) return rc_;                           \
        CK((s), (call));                               \
        rc_ = stat_end((s), (st));                     \
        if (rc_) return rc_;                           \
    } while (0)

// row blocks of the D~^T stream launch (and of the partial rows it leaves)
int t2_blocks(int64_t ns, int64_t ld, int prec)
{
    const int64_t nch = ld / (prec == IRL_FP64 ? 2 : 4);
    const int ntiles = (int)((nch + 64 * 16 - 1) / (64 * 16));
    int nblk = kStreamBlocks / ntiles;
    if (nblk < 1) nblk = 1;
    if (nblk > (ns + 3) / 4) nblk = (int)((ns + 3) / 4);
    return nblk;
}

// Z, E and the gradient from psi: H psi -> reductions -> grad_full = 2 D~^T (H psi - E psi) / Z.
// With the factored Jacobian the gradient is its backward product; with an FP64
// copy of D~ it streams that copy (and leaves D~^T psi in y as a diagnostic);
// without either, and with the network at hand (nqs), it is recomputed from
// theta in FP64; only a caller-set FP32 D~ falls back to the FP32 stream.
int energy_and_gradient(irl_system *s, void *ws, const WsLayout &L, hipStream_t st,
                        const irl_nqs_desc *nqs = nullptr)
{
    double *psi = ws_ptr<double>(ws, L.off_psi), *hpsi = ws_ptr<double>(ws, L.off_hpsi);
    TIMED(s, IRL_STAT_HAM_APPLY, st, launch_ham_apply(s, psi, hpsi, st));
    TIMED(s, IRL_STAT_ENERGY, st, launch_energy_reduce(L, ws, st));
    WsScalars *sc = ws_ptr<WsScalars>(ws, L.off_scal);
    const int prec = (L.flags & IRL_WS_FP64) ? IRL_FP64 : IRL_FP32;
    int nblk = 1;
    double *y = ws_ptr<double>(ws, L.off_y);
    if (L.flags & IRL_WS_FACTORED) {
        nblk = fac_vjp_blocks(s, L);
        TIMED(s, IRL_STAT_ENERGY, st, launch_fac_vjp(s, L, ws, hpsi, nullptr, &sc->E_el, 1, nblk, st));
        y = nullptr;
    } else if (prec == IRL_FP32 && nqs) {
        nblk = t2_blocks(L.ns, L.ld32, IRL_FP32);
        TIMED(s, IRL_STAT_ENERGY, st, launch_nqs_grad(s, nqs->V, nqs->H, nqs->theta, L, ws, nblk, st));
        y = nullptr;
    } else {
        TIMED(s, prec == IRL_FP64 ? IRL_STAT_GEMV_T : IRL_STAT_GEMV_T_LO, st,
              launch_gemv_t2(L, ws, prec, psi, hpsi, psi, &sc->E_el, &nblk, st));
    }
    TIMED(s, IRL_STAT_REDUCE, st, launch_t2_reduce(L, ws, nblk, y, ws_ptr<double>(ws, L.off_grad),
                                                   L.ncols, 2.0, &sc->Z, st));
    int rc = read_scalars(s, ws, L, st);
    if (rc) return rc;
    s->Z = s->host_scal->Z;
    s->E_el = s->host_scal->E_el;
    if (!(s->Z > 0.0) || !std::isfinite(s->E_el))
        return set_err(s, IRL_EINVAL, "psi^T psi is zero or the energy is not finite");
    return IRL_OK;
}

// connected basis (mode C): sig = D~^T psi into ws (one backward product with psi)
int connected_sigma(irl_system *s, void *ws, const WsLayout &L, hipStream_t st)
{
    const double *psi = ws_ptr<double>(ws, L.off_psi);
    double *sig = ws_ptr<double>(ws, L.off_sig);
    int nblk = 1;
    if (L.flags & IRL_WS_FACTORED) {
        nblk = fac_vjp_blocks(s, L);
        TIMED(s, IRL_STAT_GEMV_T, st, launch_fac_vjp(s, L, ws, psi, nullptr, nullptr, 0, nblk, st));
    } else {
        TIMED(s, IRL_STAT_GEMV_T, st, launch_gemv_t2(L, ws, IRL_FP64, psi, psi, nullptr, nullptr, &nblk, st));
    }
    TIMED(s, IRL_STAT_REDUCE, st, launch_t2_reduce(L, ws, nblk, sig, nullptr, L.ncols, 1.0, nullptr, st));
    return IRL_OK;
}

// the operator pair into ws yH/yS (internal, ldv long); zero_v0: apply to (0, v[1:])
int apply_internal(irl_system *s, void *ws, const WsLayout &L, const double *v, double *yH,
                   double *yS, int prec, hipStream_t st, int zero_v0 = 0)
{
    double *w = ws_ptr<double>(ws, L.off_w), *u = ws_ptr<double>(ws, L.off_u);
    if (prec == IRL_FP64 && (L.flags & IRL_WS_FACTORED) && s->vmc && s->vmc_rows > 0) {
        // sampled operator on the drawn rows only (gathered contiguously by irl_vmc_sample)
        const FacRows R{ws_ptr<uint64_t>(ws, L.off_ckeys), s->vmc_rows, ws_ptr<double>(ws, L.off_cpsi),
                        ws_ptr<double>(ws, L.off_cfac)};
        TIMED(s, IRL_STAT_GEMV, st, launch_fac_jvp_rows(s, L, R, v, zero_v0, w, st));
        TIMED(s, IRL_STAT_VMC, st, launch_vmc_diag_rows(L, ws, s->vmc_rows, w, u, st));
        const int nb = fac_row_blocks_n(s, s->vmc_rows, L.hfac);
        TIMED(s, IRL_STAT_GEMV_T, st, launch_fac_vjp_rows(s, L, ws, R, w, u, nullptr, 0, nb, st));
        TIMED(s, IRL_STAT_REDUCE, st, launch_t2_reduce(L, ws, nb, yS, yH, L.ncols, 1.0, nullptr, st));
        return IRL_OK;
    }
    if (prec == IRL_FP64 && (L.flags & IRL_WS_FACTORED)) {
        // factored Jacobian: forward product, H, both backward products in one pass
        TIMED(s, IRL_STAT_GEMV, st, launch_fac_jvp(s, L, ws, v, zero_v0, w, st));
        if (s->vmc)
            TIMED(s, IRL_STAT_VMC, st, launch_vmc_diag(L, ws, w, u, 1, st));
        else
            TIMED(s, IRL_STAT_HAM_APPLY, st, launch_ham_apply(s, w, u, st));
        const int nb = fac_vjp_blocks(s, L);
        TIMED(s, IRL_STAT_GEMV_T, st, launch_fac_vjp(s, L, ws, w, u, nullptr, 0, nb, st));
        TIMED(s, IRL_STAT_REDUCE, st, launch_t2_reduce(L, ws, nb, yS, yH, L.ncols, 1.0, nullptr, st));
        return IRL_OK;
    }
    TIMED(s, prec == IRL_FP64 ? IRL_STAT_GEMV : IRL_STAT_GEMV_LO, st, launch_gemv_rows(L, ws, prec, v, w, zero_v0, st));
    if (s->vmc)
        TIMED(s, IRL_STAT_VMC, st, launch_vmc_diag(L, ws, w, u, 1, st));
    else
        TIMED(s, IRL_STAT_HAM_APPLY, st, launch_ham_apply(s, w, u, st));
    int nblk = 1;
    TIMED(s, prec == IRL_FP64 ? IRL_STAT_GEMV_T : IRL_STAT_GEMV_T_LO, st, launch_gemv_t2(L, ws, prec, w, u, nullptr, nullptr, &nblk, st));
    TIMED(s, IRL_STAT_REDUCE, st, launch_t2_reduce(L, ws, nblk, yS, yH, L.ncols, 1.0, nullptr, st));
    return IRL_OK;
}

// nb operator pairs at once: W = D~ V (one D~ pass), U_q = H W_q, (YS, YH) = D~^T (W, U)
// (one D~ pass); V columns stride ldv_in, outputs stride ldy
int apply_block_internal(irl_system *s, void *ws, const WsLayout &L, const double *V, int64_t ldv_in, int nb,
                         double *YH, double *YS, int64_t ldy, int prec, hipStream_t st, int zero_v0 = 0)
{
    if (prec == IRL_FP64 && (L.flags & IRL_WS_FACTORED)) {
        // factored Jacobian: the products read d (H values per row) instead of a
        // D~ row, and H is applied per vector anyway, so the block is nb
        // single-vector applies (d read twice per vector)
        for (int q = 0; q < nb; ++q) {
            const int rc = apply_internal(s, ws, L, V + (int64_t)q * ldv_in, YH + (int64_t)q * ldy,
                                          YS + (int64_t)q * ldy, prec, st, zero_v0);
            if (rc) return rc;
        }
        return IRL_OK;
    }
    double *W = ws_ptr<double>(ws, L.off_w), *U = ws_ptr<double>(ws, L.off_u);
    TIMED(s, prec == IRL_FP64 ? IRL_STAT_GEMV : IRL_STAT_GEMV_LO, st,
          launch_gemv_rows_multi(L, ws, prec, V, ldv_in, nb, zero_v0, W, st));
    if (s->vmc) {
        TIMED(s, IRL_STAT_VMC, st, launch_vmc_diag(L, ws, W, U, nb, st));
    } else {
        for (int q = 0; q < nb; ++q)
            TIMED(s, IRL_STAT_HAM_APPLY, st, launch_ham_apply(s, W + (int64_t)q * L.ns, U + (int64_t)q * L.ns, st));
    }
    int nblk = 1;
    TIMED(s, prec == IRL_FP64 ? IRL_STAT_GEMV_T : IRL_STAT_GEMV_T_LO, st,
          launch_gemv_t2_multi(L, ws, prec, nb, W, U, &nblk, st));
    TIMED(s, IRL_STAT_REDUCE, st, launch_t2_reduce_multi(L, ws, nblk, nb, YS, YH, ldy, st));
    return IRL_OK;
}

int check_prec(irl_system *s, int prec)
{
    if (prec == IRL_FP64 && !s->ws_has64)
        return set_err(s, IRL_ESTATE, "workspace holds neither an FP64 copy of D~ nor the factored Jacobian");
    if (prec == IRL_FP32 && !s->ws_has32)
        return set_err(s, IRL_ESTATE, "workspace holds no FP32 copy of D~");
    if (prec != IRL_FP64 && prec != IRL_FP32) return set_err(s, IRL_EINVAL, "bad precision");
    return IRL_OK;
}

}  // namespace

namespace irl {

WsLayout make_layout(int64_t ns, int64_t ncols, uint32_t flags, int V, int64_t fullA, int64_t fullB)
{
    WsLayout L;
    L.ns = ns;
    L.ncols = ncols;
    L.flags = flags;
    if ((flags & IRL_WS_FACTORED) && V > 0 && (ncols - 1 - V) > 0 && (ncols - 1 - V) % (V + 1) == 0)
        L.hfac = (int)((ncols - 1 - V) / (V + 1));
    const int64_t ld = (int64_t)align_up((size_t)ncols, 32);
    L.ld64 = L.ld32 = L.ldv = ld;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = align_up(off + bytes, 256);
        return o;
    };
    L.off_scal = take(sizeof(WsScalars));
    L.off_d64 = take((flags & IRL_WS_FP64) ? (size_t)ns * ld * sizeof(double) : 0);
    L.off_d32 = take((flags & IRL_WS_FP32) ? (size_t)ns * ld * sizeof(float) : 0);
    const size_t nvec = (size_t)layout_vectors(L);   // vectors per w/u/yH/yS region
    L.off_psi = take((size_t)ns * 8);
    L.off_hpsi = take((size_t)ns * 8);
    L.off_w = take((size_t)ns * 8 * nvec);
    L.off_u = take((size_t)ns * 8 * nvec);
    L.off_grad = take((size_t)ld * 8);
    L.off_yh = take((size_t)ld * 8 * nvec);
    L.off_ys = take((size_t)ld * 8 * nvec);
    L.off_y = take((size_t)ld * 8);
    L.off_r = take((size_t)ld * 8);
    L.off_vconv = take((size_t)ld * 8 * nvec);
    L.off_part = take((size_t)kStreamBlocks * 2 * ld * 8);
    L.off_part2 = take((size_t)kReduceGroups * 2 * ld * 8 * nvec);
    L.off_red = take((size_t)kScalarParts * 4 * 8);
    L.off_kry0 = take((size_t)kBasisCols * ld * 8);
    L.off_kry1 = take((size_t)kBasisCols * ld * 8);
    L.off_img0 = take((size_t)kBasisCols * ld * 8);
    L.off_img1 = take((size_t)kBasisCols * ld * 8);
    L.off_hy = take((size_t)ld * 8);
    L.off_fac = take((flags & IRL_WS_FACTORED) ? (size_t)ns * (size_t)L.hfac * 8 : 0);
    L.off_sig = take((size_t)ld * 8);
    L.off_q = take((size_t)ns * 8);
    L.off_warm = take((size_t)ld * 8);
    const bool gather = (flags & IRL_WS_SAMPLED) && (flags & IRL_WS_FACTORED) && L.hfac > 0;
    L.off_ckeys = take(gather ? (size_t)ns * 8 : 0);
    L.off_cpsi = take(gather ? (size_t)ns * 8 : 0);
    L.off_cq = take(gather ? (size_t)ns * 8 : 0);
    L.off_cel = take(gather ? (size_t)ns * 8 : 0);
    L.off_crow = take(gather ? (size_t)ns * 8 : 0);
    L.off_cfac = take(gather ? (size_t)ns * (size_t)L.hfac * 8 : 0);
    if ((flags & IRL_WS_FACTORED) && L.hfac > 0 && fullA > 0 && fullA * fullB == ns)
        L.kf_S = fac_full_ranges(fullA, fullB, V / 2, L.hfac);
    L.total = off;
    return L;
}

// Adam update of theta from the gradient (lanczos.hip)
hipError_t launch_adam(double *theta, const double *g, double *m, double *v, int64_t P, double lr, double b1,
                       double b2, double eps, int64_t t, hipStream_t st);

}  // namespace irl

namespace {

// One implicitly restarted Lanczos solve of the centred operator at precision
// prec, from a random start vector or from start (device, ldv doubles).  On
// return the unit Ritz vector is in ws y.
struct SolveOut {
    double lam = 0, resid_est = 0, resid_explicit = 0, gap = 0, normT = 0, c0 = 0, tol_used = 0;
    int n_apply = 0, n_restart = 0, converged = 0, n_graph = 0;
};

// ---- captured Lanczos cycles -------------------------------------------------
// On operators small enough that the solve is launch-bound (no in-cycle tests),
// a whole cycle -- the m - j0 applies with their Lanczos steps and the Ritz /
// restart-shift kernel, preceded by the basis restart for the restart cycles --
// is captured once into a HIP graph and replayed: the first cycle (basis 0) and
// the restart cycles from basis 0 and from basis 1.  The seeds of the captured
// kernels are the solve's seed; the per-cycle seed is derived on the device from
// the restart count, so a replay runs exactly the eager arithmetic.  The graphs
// hold the workspace's pointers and every launch shape of the apply, so they are
// keyed on all of them and rebuilt when any changes (one entry per precision).
struct CycleKey {
    void *ws = nullptr;
    size_t total = 0;
    int64_t ns = 0, ncols = 0;
    uint32_t flags = 0;
    int m = 0, k = 0, mode = 0, prec = 0, ham_kernel = -1;
    uint64_t seed = 0;
    bool vmc = false;
    int64_t vmc_rows = 0;
    const void *hptr = nullptr;
    int32_t tune_lut = 0, tune_pull = 0, tune_waves = 0;   // launch shapes recorded in the graph
    bool operator==(const CycleKey &o) const
    {
        return ws == o.ws && total == o.total && ns == o.ns && ncols == o.ncols && flags == o.flags && m == o.m &&
               k == o.k && mode == o.mode && prec == o.prec && ham_kernel == o.ham_kernel && seed == o.seed &&
               vmc == o.vmc && vmc_rows == o.vmc_rows && hptr == o.hptr && tune_lut == o.tune_lut &&
               tune_pull == o.tune_pull && tune_waves == o.tune_waves;
    }
};

struct CycleEntry {
    CycleKey key;
    bool valid = false, failed = false;
    hipGraphExec_t exec[3] = {nullptr, nullptr, nullptr};   // first cycle, restart from basis 0, from basis 1
};

struct CycleGraphs {
    CycleEntry e[2];   // by precision
};

void drop_entry(CycleEntry &c)
{
    for (auto &x : c.exec)
        if (x) {
            (void)hipGraphExecDestroy(x);
            x = nullptr;
        }
    c.valid = false;
    c.failed = false;
}

void free_cycle_graphs(irl_system *s)
{
    if (!s || !s->cycle_graphs) return;
    CycleGraphs *g = static_cast<CycleGraphs *>(s->cycle_graphs);
    for (auto &c : g->e) drop_entry(c);
    delete g;
    s->cycle_graphs = nullptr;
}

CycleEntry *cycle_entry(irl_system *s, const CycleKey &key)
{
    if (!s->cycle_graphs) s->cycle_graphs = new CycleGraphs();
    CycleEntry &c = static_cast<CycleGraphs *>(s->cycle_graphs)->e[key.prec == IRL_FP64 ? 0 : 1];
    if (!c.valid || !(c.key == key)) {
        drop_entry(c);
        c.key = key;
        c.valid = true;
    }
    return c.failed ? nullptr : &c;
}

int apply_internal(irl_system *s, void *ws, const WsLayout &L, const double *v, double *yH, double *yS, int prec,
                   hipStream_t st, int zero_v0);

// capture cycle `kind` (0: first cycle from basis 0; 1, 2: restart from basis
// kind - 1, then the cycle from k on the other basis) on the library's capture
// stream; false if any launch or the capture itself fails (eager path then)
bool capture_cycle(irl_system *s, void *ws, const WsLayout &L, const irl_solver_opts &o, int prec, int m,
                   int k, int kind, hipGraphExec_t *out)
{
    if (!s->capture_stream && hipStreamCreateWithFlags(&s->capture_stream, hipStreamNonBlocking) != hipSuccess) {
        s->capture_stream = nullptr;
        return false;
    }
    hipStream_t cs = s->capture_stream;
    hipError_t eb = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (eb != hipSuccess) {
        (void)hipGetLastError();
        s->err = std::string("graph capture not started: ") + hipGetErrorString(eb);
        return false;
    }
    const int split = (prec == IRL_FP32) ? 1 : 0;
    double *Vb[2] = {ws_ptr<double>(ws, L.off_kry0), ws_ptr<double>(ws, L.off_kry1)};
    double *Ib[2] = {ws_ptr<double>(ws, L.off_img0), ws_ptr<double>(ws, L.off_img1)};
    double *yH = ws_ptr<double>(ws, L.off_yh), *yS = ws_ptr<double>(ws, L.off_ys);
    bool ok = true;
    std::string why;
    int cur = 0, j0 = 0;
    if (kind > 0) {
        cur = kind - 1;
        ok = launch_restart_basis(L, ws, Vb[cur], Vb[1 - cur], Ib[cur], Ib[1 - cur], m, k, o.mode, o.seed, cs) ==
             hipSuccess;
        if (!ok) why = "restart kernel";
        cur = 1 - cur;
        j0 = k;
    }
    for (int j = j0; ok && j < m; ++j) {
        ok = apply_internal(s, ws, L, Vb[cur] + (int64_t)j * L.ldv, yH, yS, prec, cs, split) == IRL_OK;
        if (!ok) {
            why = "operator apply (" + s->err + ")";
            break;
        }
        ok = launch_lanczos_step(L, ws, Vb[cur], Ib[cur], j, o.mode, split, o.seed, cs) == hipSuccess;
        if (!ok) why = "Lanczos step";
    }
    if (ok && launch_ritz(L, ws, m, k, cs) != hipSuccess) {
        ok = false;
        why = "Ritz kernel";
    }
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(cs, &g);
    if (ok && (e != hipSuccess || !g)) {
        ok = false;
        why = std::string("end of capture: ") + hipGetErrorString(e);
    }
    if (ok) {
        const hipError_t ei = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
        if (ei != hipSuccess) {
            ok = false;
            why = std::string("instantiation: ") + hipGetErrorString(ei);
        }
    }
    if (g) (void)hipGraphDestroy(g);
    if (!ok) {
        *out = nullptr;
        (void)hipGetLastError();
        s->err = "graph capture failed (launching the cycle instead): " + why;
    }
    return ok;
}

int irl_solve(irl_system *s, void *ws, const WsLayout &L, const irl_solver_opts &o, int prec,
              const double *start, SolveOut &out, hipStream_t st)
{
    const int64_t dim = (o.mode != IRL_MODE_P) ? L.ncols : L.ncols - 1;
    const int m = (int)std::min<int64_t>(o.m, dim);
    const int k = std::min(o.k_keep, m - 1);
    if (m < 2 || k < 1) return set_err(s, IRL_EINVAL, "problem dimension too small for the Krylov space");
    const double u_op = (prec == IRL_FP64) ? 1.1102230246251565e-16 : 5.960464477539063e-08;
    // reduced-precision operator: psi row/column of H~' from the FP64 gradient (split form)
    const int split = (prec == IRL_FP32) ? 1 : 0;
    double *Vb[2] = {ws_ptr<double>(ws, L.off_kry0), ws_ptr<double>(ws, L.off_kry1)};
    double *Ib[2] = {ws_ptr<double>(ws, L.off_img0), ws_ptr<double>(ws, L.off_img1)};
    int cur = 0;
    double *yH = ws_ptr<double>(ws, L.off_yh), *yS = ws_ptr<double>(ws, L.off_ys);
    double *y = ws_ptr<double>(ws, L.off_y), *rv = ws_ptr<double>(ws, L.off_r);
    double *hy = ws_ptr<double>(ws, L.off_hy);
    int rc;
    TIMED(s, IRL_STAT_RITZ, st, launch_reset_solve(L, ws, st));
    if (start) {
        TIMED(s, IRL_STAT_RITZ, st, launch_copy(Vb[0], start, L.ldv, st));
    } else {
        TIMED(s, IRL_STAT_RITZ, st, launch_start_vector(Vb[0], L.ncols, L.ldv, o.mode, o.seed, st));
    }
    int j0 = 0, n_apply = 0, n_restart = 0;
    bool converged = false;
    double tol_eff = o.tol;
    // Early checks: on large operators the Ritz pair of T_j is also tested after
    // every Lanczos step inside a cycle (an m-step cycle otherwise runs to the end
    // before its convergence test).  A check costs a few small kernels and one
    // stream synchronisation, negligible next to an apply that streams >= 256 MB.
    const double apply_bytes = 2.0 * (double)L.ns * (double)L.ldv * (prec == IRL_FP64 ? 8.0 : 4.0);
    const int stride = (o.flags & IRL_STEP_FULL_CYCLES) ? 0 : (apply_bytes >= 2.56e8 ? kCheckStride : 0);
    // graph replay of whole cycles (launch-bound solves without in-cycle tests)
    CycleEntry *cg = nullptr;
    if ((o.flags & IRL_STEP_GRAPH) && stride == 0 && !s->stats_on) {
        CycleKey key;
        key.ws = ws;
        key.total = L.total;
        key.ns = L.ns;
        key.ncols = L.ncols;
        key.flags = L.flags;
        key.m = m;
        key.k = k;
        key.mode = o.mode;
        key.prec = prec;
        key.ham_kernel = s->ham_kernel;
        key.seed = o.seed;
        key.vmc = s->vmc;
        key.vmc_rows = s->vmc_rows;
        key.hptr = s->d.scb ? (const void *)s->d.sval : (const void *)s->d.hptr;
        key.tune_lut = s->tune_lut_blocks;
        key.tune_pull = s->tune_pull_blocks;
        key.tune_waves = s->tune_pull_waves;
        cg = cycle_entry(s, key);
    }
    int pending = -1;   // restart not yet launched: from basis `pending` (graph replay)
    for (;;) {
        int mc = m;   // size of the tridiagonal tested at the end of this pass
        bool early = false;
        const int kind = pending >= 0 ? 1 + pending : (j0 == 0 && cur == 0 ? 0 : -1);
        if (cg && kind >= 0 && !cg->exec[kind] && !capture_cycle(s, ws, L, o, prec, m, k, kind, &cg->exec[kind])) {
            cg->failed = true;
            cg = nullptr;
        }
        if (!cg && pending >= 0) {
            // capture failed after a restart was deferred: launch it eagerly
            TIMED(s, IRL_STAT_RITZ, st,
                  launch_restart_basis(L, ws, Vb[pending], Vb[1 - pending], Ib[pending], Ib[1 - pending], m, k,
                                       o.mode, o.seed, st));
            pending = -1;
        }
        if (cg && kind >= 0) {
            CK(s, hipGraphLaunch(cg->exec[kind], st));
            n_apply += m - j0;
            ++out.n_graph;
            pending = -1;
        } else {
        for (int j = j0; j < m; ++j) {
            rc = apply_internal(s, ws, L, Vb[cur] + (int64_t)j * L.ldv, yH, yS, prec, st, split);
            if (rc) return rc;
            ++n_apply;
            TIMED(s, IRL_STAT_LANCZOS, st,
                  launch_lanczos_step(L, ws, Vb[cur], Ib[cur], j, o.mode, split,
                                      o.seed, st));
            if (stride && j + 1 < m && j + 1 >= 2 && (j + 1 - j0) % stride == 0) {
                TIMED(s, IRL_STAT_RITZ, st, launch_ritz(L, ws, j + 1, 0, st));
                rc = read_scalars(s, ws, L, st);
                if (rc) return rc;
                const double tq = std::max(o.tol, 64.0 * u_op * s->host_scal->normT);
                if (s->host_scal->resid_est <= tq && std::isfinite(s->host_scal->lam)) {
                    mc = j + 1;
                    early = true;
                    break;
                }
            }
        }
        if (!early) TIMED(s, IRL_STAT_RITZ, st, launch_ritz(L, ws, m, k, st));
        }
        rc = read_scalars(s, ws, L, st);
        if (rc) return rc;
        const WsScalars &hs = *s->host_scal;
        tol_eff = std::max(o.tol, 64.0 * u_op * hs.normT);
        out.lam = hs.lam;
        out.resid_est = hs.resid_est;
        out.gap = hs.gap;
        out.normT = hs.normT;
        if (!std::isfinite(hs.lam)) return set_err(s, IRL_EINVAL, "non-finite Ritz value (check theta and D~)");
        if (hs.resid_est <= tol_eff) {
            // explicit residual: the Ritz vector's image is the same combination of
            // the stored images H~' v_j, so no further operator apply is needed
            TIMED(s, IRL_STAT_RITZ, st, launch_ritz_vector(L, ws, Vb[cur], Ib[cur], mc, y, hy, st));
            TIMED(s, IRL_STAT_RITZ, st, launch_residual_image(L, ws, y, hy, rv, o.mode, st));
            rc = read_scalars(s, ws, L, st);
            if (rc) return rc;
            out.resid_explicit = std::sqrt(s->host_scal->resid2);
            const double tol_explicit = std::max(tol_eff, 1024.0 * u_op * hs.normT);
            if (out.resid_explicit <= tol_explicit) {
                converged = true;
                break;
            }
        }
        if (early) {
            // explicit test failed on an early candidate: continue the cycle
            j0 = mc;
            continue;
        }
        if (n_restart >= o.max_restarts) break;
        if (cg) {
            pending = cur;   // the restart opens the next captured cycle
        } else {
            TIMED(s, IRL_STAT_RITZ, st,
                  launch_restart_basis(L, ws, Vb[cur], Vb[1 - cur], Ib[cur], Ib[1 - cur], m, k, o.mode,
                                       o.seed, st));
        }
        cur = 1 - cur;
        j0 = k;
        ++n_restart;
    }
    if (!converged) {
        // report the current Ritz pair
        TIMED(s, IRL_STAT_RITZ, st, launch_ritz(L, ws, m, 0, st));
        TIMED(s, IRL_STAT_RITZ, st, launch_ritz_vector(L, ws, Vb[cur], Ib[cur], m, y, hy, st));
        TIMED(s, IRL_STAT_RITZ, st, launch_residual_image(L, ws, y, hy, rv, o.mode, st));
        rc = read_scalars(s, ws, L, st);
        if (rc) return rc;
        out.resid_explicit = std::sqrt(s->host_scal->resid2);
    }
    out.c0 = s->host_scal->c0;
    out.n_apply = n_apply;
    out.n_restart = n_restart;
    out.converged = converged ? 1 : 0;
    out.tol_used = tol_eff;
    return IRL_OK;
}

// Thick-restart block Lanczos solve (opts.block = nb >= 2 vectors per operator
// pass); same outputs and convergence test as irl_solve.  m counts basis columns.
int irl_solve_block(irl_system *s, void *ws, const WsLayout &L, const irl_solver_opts &o, int prec,
                    SolveOut &out, hipStream_t st)
{
    const int nb = o.block;
    if (!(L.flags & IRL_WS_BLOCK)) return set_err(s, IRL_EINVAL, "block solves need a workspace with IRL_WS_BLOCK");
    if (nb < 2 || nb > kMaxBlock) return set_err(s, IRL_EINVAL, "block must be in [2, 8]");
    const int64_t dim = (o.mode == IRL_MODE_A) ? L.ncols : L.ncols - 1;
    const int m = (int)std::min<int64_t>(std::min(o.m, kMaxKrylov), dim);
    const int k = std::min(o.k_keep, m - nb);
    if (m < 2 * nb || k < 1) return set_err(s, IRL_EINVAL, "block solve needs 2 * block <= m and 1 <= k_keep <= m - block");
    const double u_op = (prec == IRL_FP64) ? 1.1102230246251565e-16 : 5.960464477539063e-08;
    const int split = (prec == IRL_FP32) ? 1 : 0;
    double *Vb[2] = {ws_ptr<double>(ws, L.off_kry0), ws_ptr<double>(ws, L.off_kry1)};
    double *Ib[2] = {ws_ptr<double>(ws, L.off_img0), ws_ptr<double>(ws, L.off_img1)};
    int cur = 0;
    double *yH = ws_ptr<double>(ws, L.off_yh), *yS = ws_ptr<double>(ws, L.off_ys);
    double *y = ws_ptr<double>(ws, L.off_y), *rv = ws_ptr<double>(ws, L.off_r);
    double *hy = ws_ptr<double>(ws, L.off_hy);
    int rc;
    TIMED(s, IRL_STAT_RITZ, st, launch_reset_solve(L, ws, st));
    TIMED(s, IRL_STAT_RITZ, st, launch_block_start(L, ws, Vb[0], nb, o.mode, o.seed, st));
    int sz = 0, n_apply = 0, n_restart = 0;
    bool converged = false;
    double tol_eff = o.tol;
    for (;;) {
        // operator on the pending block, then one block step: basis grows to sz + nb
        rc = apply_block_internal(s, ws, L, Vb[cur] + (int64_t)sz * L.ldv, L.ldv, nb, yH, yS, L.ldv, prec, st,
                                  split);
        if (rc) return rc;
        n_apply += nb;
        TIMED(s, IRL_STAT_LANCZOS, st,
              launch_block_step(L, ws, Vb[cur], Ib[cur], sz, nb, o.mode, split,
                                o.seed + 0x100000001b3ull * (uint64_t)(n_restart + 1), st));
        sz += nb;
        TIMED(s, IRL_STAT_RITZ, st, launch_block_ritz(L, ws, sz, nb, st));
        rc = read_scalars(s, ws, L, st);
        if (rc) return rc;
        const WsScalars &hs = *s->host_scal;
        tol_eff = std::max(o.tol, 64.0 * u_op * hs.normT);
        out.lam = hs.lam;
        out.resid_est = hs.resid_est;
        out.gap = hs.gap;
        out.normT = hs.normT;
        if (!std::isfinite(hs.lam)) return set_err(s, IRL_EINVAL, "non-finite Ritz value (check theta and D~)");
        if (hs.resid_est <= tol_eff) {
            TIMED(s, IRL_STAT_RITZ, st, launch_ritz_vector(L, ws, Vb[cur], Ib[cur], sz, y, hy, st));
            TIMED(s, IRL_STAT_RITZ, st, launch_residual_image(L, ws, y, hy, rv, o.mode, st));
            rc = read_scalars(s, ws, L, st);
            if (rc) return rc;
            out.resid_explicit = std::sqrt(s->host_scal->resid2);
            if (out.resid_explicit <= std::max(tol_eff, 1024.0 * u_op * hs.normT)) {
                converged = true;
                break;
            }
        }
        if (sz + nb > m) {
            if (n_restart >= o.max_restarts) break;
            TIMED(s, IRL_STAT_RITZ, st,
                  launch_block_restart(L, ws, Vb[cur], Vb[1 - cur], Ib[cur], Ib[1 - cur], sz, k, nb, st));
            cur = 1 - cur;
            sz = k;
            ++n_restart;
        }
    }
    if (!converged) {
        TIMED(s, IRL_STAT_RITZ, st, launch_block_ritz(L, ws, sz, nb, st));
        TIMED(s, IRL_STAT_RITZ, st, launch_ritz_vector(L, ws, Vb[cur], Ib[cur], sz, y, hy, st));
        TIMED(s, IRL_STAT_RITZ, st, launch_residual_image(L, ws, y, hy, rv, o.mode, st));
        rc = read_scalars(s, ws, L, st);
        if (rc) return rc;
        out.resid_explicit = std::sqrt(s->host_scal->resid2);
    }
    out.c0 = s->host_scal->c0;
    out.n_apply = n_apply;
    out.n_restart = n_restart;
    out.converged = converged ? 1 : 0;
    out.tol_used = tol_eff;
    return IRL_OK;
}

}  // namespace

extern "C" {

const char *irl_last_error(const irl_system *sys)
{
    return sys ? sys->err.c_str() : g_create_err.c_str();
}

void irl_solver_opts_default(irl_solver_opts *o)
{
    if (!o) return;
    o->m = 20;
    o->k_keep = 1;
    o->tol = 1e-12;
    o->max_restarts = 300;
    o->precision = IRL_FP64;
    o->mode = IRL_MODE_A;
    o->seed = 0;
    o->flags = 0;
    o->block = 0;
}

int irl_system_create(const irl_system_desc *d, void *stream, irl_system **out)
{
    if (!out) return set_err(nullptr, IRL_EINVAL, "out is NULL");
    *out = nullptr;
    if (!d) return set_err(nullptr, IRL_EINVAL, "desc is NULL");
    const int n = d->n_orb, na = d->n_alpha, nb = d->n_beta;
    if (n < 1 || n > 32) return set_err(nullptr, IRL_EINVAL, "n_orb must be in [1, 32]");
    if (na < 0 || na > n || nb < 0 || nb > n)
        return set_err(nullptr, IRL_EINVAL, "electron counts out of range");
    if (!d->h || !d->g) return set_err(nullptr, IRL_EINVAL, "integrals are NULL");
    // symmetry of the integrals
    double gmax = 1.0;
    const size_t n2 = (size_t)n * n, n4 = n2 * n2;
    for (size_t i = 0; i < n2; ++i) gmax = std::max(gmax, std::fabs(d->h[i]));
    for (size_t i = 0; i < n4; ++i) {
        if (!std::isfinite(d->g[i])) return set_err(nullptr, IRL_EINVAL, "g is not finite");
        gmax = std::max(gmax, std::fabs(d->g[i]));
    }
    const double stol = 1e-12 * gmax;
    for (int p = 0; p < n; ++p)
        for (int q = 0; q < n; ++q)
            if (!(std::fabs(d->h[p * n + q] - d->h[q * n + p]) <= stol))
                return set_err(nullptr, IRL_EINVAL, "h is not symmetric");
    auto G = [&](int p, int q, int r, int s_) { return d->g[(((size_t)p * n + q) * n + r) * n + s_]; };
    for (int p = 0; p < n; ++p)
        for (int q = 0; q < n; ++q)
            for (int r = 0; r < n; ++r)
                for (int s_ = 0; s_ < n; ++s_) {
                    double v = G(p, q, r, s_);
                    if (!(std::fabs(v - G(q, p, r, s_)) <= stol && std::fabs(v - G(p, q, s_, r)) <= stol &&
                          std::fabs(v - G(r, s_, p, q)) <= stol))
                        return set_err(nullptr, IRL_EINVAL, "g is not 8-fold symmetric");
                }

    irl_system *s = new irl_system();
    s->n = n;
    s->na = na;
    s->nb = nb;
    s->e_core = d->e_core;
    s->sys_flags = d->flags;
    hipStream_t st = (hipStream_t)stream;
    (void)hipGetDevice(&s->device);
    {
        const hipError_t e = noalloc_scratch_setup(s->device);
        if (e != hipSuccess) {
            free_system(s);
            return set_err(nullptr, IRL_EDEVICE, std::string("scratch symbol address: ") + hipGetErrorString(e));
        }
    }
    const int64_t cA = binom_host(n, na), cB = binom_host(n, nb);
    std::vector<uint64_t> keys;
    bool full = (d->dets == nullptr);
    if (!full) {
        if (d->n_dets <= 0) { free_system(s); return set_err(nullptr, IRL_EINVAL, "empty determinant set"); }
        keys.assign(d->dets, d->dets + d->n_dets);
        std::sort(keys.begin(), keys.end());
        for (size_t i = 0; i < keys.size(); ++i) {
            uint32_t al = (uint32_t)keys[i], be = (uint32_t)(keys[i] >> 32);
            if (i > 0 && keys[i] == keys[i - 1]) { free_system(s); return set_err(nullptr, IRL_EINVAL, "duplicate determinant keys"); }
            if (keys[i] == kEmptyKey) { free_system(s); return set_err(nullptr, IRL_EINVAL, "key 2^64 - 1 is reserved"); }
            if ((n < 32 && ((al >> n) || (be >> n))) || __builtin_popcount(al) != na ||
                __builtin_popcount(be) != nb) {
                free_system(s);
                return set_err(nullptr, IRL_EINVAL, "determinant with wrong electron count or orbital outside n");
            }
        }
        if ((int64_t)keys.size() == cA * cB && n <= 24) full = true;   // the set is the full space
    }
    if (full && n > 24) { free_system(s); return set_err(nullptr, IRL_EINVAL, "full space needs n_orb <= 24"); }
    s->ns = full ? cA * cB : (int64_t)keys.size();
    if (s->ns >= (int64_t)1 << 31) { free_system(s); return set_err(nullptr, IRL_EINVAL, "more than 2^31 - 1 determinants"); }
    s->full = full;
    s->nA = full ? cA : 0;
    s->nB = full ? cB : 0;
    const bool want_hash = !full || (d->flags & IRL_SYS_FORCE_HASH);
    // selected sets: rows sharing a beta string form one contiguous block of the
    // sorted keys (beta-major order); a direct beta -> block table plus a binary
    // search over the block's alpha strings replaces the hash on the apply path
    const bool want_blocks = !full && n <= 24 && !(d->flags & IRL_SYS_FORCE_HASH);
    s->ham_kernel = want_blocks ? 3 : (want_hash ? 0 : 1);
    s->lookup = want_blocks ? kLkBlocks : (want_hash ? kLkHash : kLkRanks);
    std::vector<int32_t> bidx, bstart, aidx, astart, arow;
    std::vector<uint32_t> abeta;
    if (want_blocks) {
        bidx.assign((size_t)1 << n, -1);
        for (size_t i = 0; i < keys.size(); ++i) {
            uint32_t be = (uint32_t)(keys[i] >> 32);
            if (i == 0 || be != (uint32_t)(keys[i - 1] >> 32)) {
                bidx[be] = (int32_t)bstart.size();
                bstart.push_back((int32_t)i);
            }
        }
        s->d.nblocks = (int64_t)bstart.size();
        bstart.push_back((int32_t)keys.size());
        // alpha-major order: a stable sort of the rows by alpha string keeps each
        // alpha block in beta order
        arow.resize(keys.size());
        for (size_t i = 0; i < keys.size(); ++i) arow[i] = (int32_t)i;
        std::stable_sort(arow.begin(), arow.end(),
                         [&](int32_t x, int32_t y) { return (uint32_t)keys[x] < (uint32_t)keys[y]; });
        aidx.assign((size_t)1 << n, -1);
        abeta.resize(keys.size());
        for (size_t i = 0; i < keys.size(); ++i) {
            const uint32_t al = (uint32_t)keys[arow[i]];
            abeta[i] = (uint32_t)(keys[arow[i]] >> 32);
            if (i == 0 || al != (uint32_t)keys[arow[i - 1]]) {
                aidx[al] = (int32_t)astart.size();
                astart.push_back((int32_t)i);
            }
        }
        astart.push_back((int32_t)keys.size());
    }

    int rc = IRL_OK;
#define AL(ptr, cnt) \
    if ((rc = dev_alloc(s, &(ptr), (cnt))) != IRL_OK) { std::string m_ = s->err; free_system(s); return set_err(nullptr, rc, m_); }
    AL(s->d.keys, (size_t)s->ns);
    AL(s->d.h, n2);
    AL(s->d.g, n4);
    AL(s->d.diag, (size_t)s->ns);
    if (full) {
        AL(s->d.rankA, (size_t)1 << n);
        AL(s->d.rankB, (size_t)1 << n);
        AL(s->d.strA, (size_t)cA);
        AL(s->d.strB, (size_t)cB);
    }
    if (want_hash) {
        uint64_t cap = 64;
        while (cap < 2 * (uint64_t)s->ns) cap <<= 1;
        s->d.hcap = cap;
        AL(s->d.hkeys, cap);
        AL(s->d.hrows, cap);
        // membership filter: ~16 bits per key, 2^16 .. 2^25 bits
        int fb = 16;
        while (fb < 25 && ((uint64_t)1 << fb) < 16 * (uint64_t)s->ns) ++fb;
        s->d.hfbits = fb;
        AL(s->d.hfilter, ((size_t)1 << fb) / 32);
    }
    if (want_blocks) {
        AL(s->d.bidx, bidx.size());
        AL(s->d.bstart, bstart.size());
        AL(s->d.aidx, aidx.size());
        AL(s->d.astart, astart.size());
        AL(s->d.arow, arow.size());
        AL(s->d.abeta, abeta.size());
    }
#undef AL
    auto fail_dev = [&](hipError_t e, const char *what) {
        std::string m_ = std::string(what) + ": " + hipGetErrorString(e);
        free_system(s);
        return set_err(nullptr, IRL_EDEVICE, m_);
    };
    hipError_t e;
    if ((e = hipMemcpyAsync(s->d.h, d->h, n2 * 8, hipMemcpyHostToDevice, st)) != hipSuccess) return fail_dev(e, "copy h");
    if ((e = hipMemcpyAsync(s->d.g, d->g, n4 * 8, hipMemcpyHostToDevice, st)) != hipSuccess) return fail_dev(e, "copy g");
    if (full) {
        if ((e = launch_enumerate_full(s->d.keys, s->d.strA, s->d.strB, s->d.rankA, s->d.rankB, n, na, nb, cA, cB, st)) != hipSuccess)
            return fail_dev(e, "enumerate");
    } else {
        if ((e = hipMemcpyAsync(s->d.keys, keys.data(), keys.size() * 8, hipMemcpyHostToDevice, st)) != hipSuccess)
            return fail_dev(e, "copy keys");
    }
    if (want_blocks) {
        if ((e = hipMemcpyAsync(s->d.bidx, bidx.data(), bidx.size() * 4, hipMemcpyHostToDevice, st)) != hipSuccess)
            return fail_dev(e, "copy block index");
        if ((e = hipMemcpyAsync(s->d.bstart, bstart.data(), bstart.size() * 4, hipMemcpyHostToDevice, st)) != hipSuccess)
            return fail_dev(e, "copy block starts");
        if ((e = hipMemcpyAsync(s->d.aidx, aidx.data(), aidx.size() * 4, hipMemcpyHostToDevice, st)) != hipSuccess ||
            (e = hipMemcpyAsync(s->d.astart, astart.data(), astart.size() * 4, hipMemcpyHostToDevice, st)) != hipSuccess ||
            (e = hipMemcpyAsync(s->d.arow, arow.data(), arow.size() * 4, hipMemcpyHostToDevice, st)) != hipSuccess ||
            (e = hipMemcpyAsync(s->d.abeta, abeta.data(), abeta.size() * 4, hipMemcpyHostToDevice, st)) != hipSuccess)
            return fail_dev(e, "copy alpha-major index");
    }
    if (want_hash)
        if ((e = launch_hash_build(s->d.keys, s->ns, s->d.hkeys, s->d.hrows, s->d.hcap, s->d.hfilter,
                                   s->d.hfbits, st)) != hipSuccess)
            return fail_dev(e, "hash build");
    if ((e = launch_diagonal(s->d.keys, s->ns, n, s->d.h, s->d.g, s->d.diag, st)) != hipSuccess)
        return fail_dev(e, "diagonal");
    if (!(d->flags & IRL_SYS_FORCE_PULL))
        if ((e = launch_product_tables(s, st)) != hipSuccess) return fail_dev(e, "product tables");
    if ((e = hipHostMalloc((void **)&s->host_scal, sizeof(WsScalars))) != hipSuccess) return fail_dev(e, "pinned scalars");
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return fail_dev(e, "system create");
    *out = s;
    return IRL_OK;
}

void irl_system_destroy(irl_system *sys) { free_system(sys); }

}  // extern "C"

namespace {

size_t sliced_bytes(int scb, int64_t ns, int64_t slots)
{
    const int64_t groups = (ns + kWave - 1) / kWave;
    return (size_t)groups * scb * 6 + (size_t)groups * kWave * scb * 2 + (size_t)scb * 8 + (size_t)slots * 10 +
           (size_t)scb * ns * 8;
}

// Stored rows in the LDS-sliced layout (every set of at most kMaxSlices slices unless
// IRL_SYS_STORE_BLOCKS): count the connections of every row per slice, order each
// window's rows by count (descending, ties by row) and group them 64 at a time
// (host), then fill the slots.
int store_sliced(irl_system *s, size_t max_bytes, size_t *bytes_needed, hipStream_t st)
{
    const int64_t ns = s->ns;
    const int scs = kSliceLog;
    const int scb = (int)((ns + ((int64_t)1 << scs) - 1) >> scs);
    const int64_t G = (ns + kWave - 1) / kWave;
    uint32_t *dcount = nullptr;
    CK(s, hipMalloc((void **)&dcount, (size_t)scb * ns * 4));
    std::vector<uint32_t> count((size_t)scb * ns);
    hipError_t e = launch_ham_count_sliced(s, scs, scb, dcount, st);
    if (e == hipSuccess) e = hipMemcpyAsync(count.data(), dcount, (size_t)scb * ns * 4, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        (void)hipFree(dcount);
        return set_err(s, IRL_EDEVICE, std::string("row counts: ") + hipGetErrorString(e));
    }
    // per slice and window: rows by count (counting sort, descending, ties by row),
    // groups of 64 lanes, slot offsets; slot[b][row] = group * 64 + lane
    std::vector<int64_t> base(scb);
    std::vector<uint32_t> gbase((size_t)scb * G), slot((size_t)scb * ns);
    std::vector<uint16_t> glen((size_t)scb * G), perm((size_t)scb * G * kWave, 0xffff);
    int64_t slots = 0, nnz = 0;
    std::vector<uint32_t> order, bucket;
    for (int b = 0; b < scb; ++b) {
        base[b] = slots;
        const uint32_t *cb = count.data() + (size_t)b * ns;
        uint64_t run = 0;
        for (int64_t w0 = 0; w0 < ns; w0 += kSellWindow) {
            const int nr = (int)std::min<int64_t>(kSellWindow, ns - w0);
            uint32_t cmax = 0;
            for (int i = 0; i < nr; ++i) cmax = std::max(cmax, cb[w0 + i]);
            bucket.assign((size_t)cmax + 2, 0u);
            for (int i = 0; i < nr; ++i) ++bucket[cmax - cb[w0 + i] + 1];
            for (uint32_t c = 1; c < cmax + 2; ++c) bucket[c] += bucket[c - 1];
            order.assign(nr, 0u);
            for (int i = 0; i < nr; ++i) order[bucket[cmax - cb[w0 + i]]++] = (uint32_t)i;
            const int64_t g0 = w0 / kWave;
            for (int k = 0; k * kWave < nr; ++k) {
                const int64_t g = g0 + k;
                // slots per lane: the longest row rounded up to 2 (two values or two
                // targets per lane and load)
                const uint32_t L = (cb[w0 + order[(size_t)k * kWave]] + 1u) & ~1u;
                if (L > 0xffffu) return (void)hipFree(dcount), set_err(s, IRL_EINVAL, "a row holds more than 65535 elements in one slice");
                gbase[(size_t)b * G + g] = (uint32_t)run;
                glen[(size_t)b * G + g] = (uint16_t)L;
                for (int l = 0; l < kWave && k * kWave + l < nr; ++l) {
                    const uint32_t i = order[(size_t)k * kWave + l];
                    perm[((size_t)b * G + g) * kWave + l] = (uint16_t)i;
                    slot[(size_t)b * ns + w0 + i] = (uint32_t)(k * kWave + l) + (uint32_t)(g0 * kWave);
                    nnz += cb[w0 + i];
                }
                run += (uint64_t)L * kWave;
                if (run > 0xffffffffull)
                    return (void)hipFree(dcount), set_err(s, IRL_EINVAL, "a slice holds more than 2^32 - 1 slots");
            }
        }
        slots += (int64_t)run;
    }
    const size_t bytes = sliced_bytes(scb, ns, slots);
    if (bytes_needed) *bytes_needed = bytes;
    if (bytes > max_bytes) {
        (void)hipFree(dcount);
        return set_err(s, IRL_ENOMEM, "stored rows need " + std::to_string(bytes) +
                                          " bytes, more than max_bytes = " + std::to_string(max_bytes));
    }
    const size_t bytes_before = s->dev_bytes;
    auto release = [&]() {
        s->dev_bytes = bytes_before;
        for (void *p : {(void *)s->d.sbase, (void *)s->d.sgbase, (void *)s->d.sglen, (void *)s->d.sperm,
                        (void *)s->d.scol, (void *)s->d.sval, (void *)s->d.spart})
            if (p) (void)hipFree(p);
        s->d.sbase = nullptr;
        s->d.sgbase = nullptr;
        s->d.sglen = nullptr;
        s->d.sperm = nullptr;
        s->d.scol = nullptr;
        s->d.sval = nullptr;
        s->d.spart = nullptr;
        s->d.sgroups = 0;
    };
    int rc;
    if ((rc = dev_alloc(s, &s->d.sbase, (size_t)scb)) != IRL_OK ||
        (rc = dev_alloc(s, &s->d.sgbase, (size_t)scb * G)) != IRL_OK ||
        (rc = dev_alloc(s, &s->d.sglen, (size_t)scb * G)) != IRL_OK ||
        (rc = dev_alloc(s, &s->d.sperm, (size_t)scb * G * kWave)) != IRL_OK ||
        (rc = dev_alloc(s, &s->d.scol, (size_t)std::max<int64_t>(slots, 1))) != IRL_OK ||
        (rc = dev_alloc(s, &s->d.sval, (size_t)std::max<int64_t>(slots, 1))) != IRL_OK ||
        (rc = dev_alloc(s, &s->d.spart, (size_t)scb * ns)) != IRL_OK) {
        (void)hipFree(dcount);
        release();
        return rc;
    }
    s->d.sgroups = (int32_t)G;
    // the slot map reuses the count buffer (scb x ns uint32)
    uint32_t *dslot = dcount;
    e = hipMemcpyAsync(dslot, slot.data(), slot.size() * 4, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(s->d.sbase, base.data(), base.size() * 8, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(s->d.sgbase, gbase.data(), gbase.size() * 4, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(s->d.sglen, glen.data(), glen.size() * 2, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(s->d.sperm, perm.data(), perm.size() * 2, hipMemcpyHostToDevice, st);
    // padding slots: target 0 (inside every slice), value 0
    if (e == hipSuccess) e = hipMemsetAsync(s->d.scol, 0, (size_t)std::max<int64_t>(slots, 1) * 2, st);
    if (e == hipSuccess) e = hipMemsetAsync(s->d.sval, 0, (size_t)std::max<int64_t>(slots, 1) * 8, st);
    if (e == hipSuccess) e = launch_ham_fill_sliced(s, scs, scb, dslot, s->d.scol, s->d.sval, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    (void)hipFree(dcount);
    if (e != hipSuccess) {
        release();
        return set_err(s, IRL_EDEVICE, std::string("stored rows: ") + hipGetErrorString(e));
    }
    s->d.scb = scb;
    s->d.scs = scs;
    s->d.hnnz = nnz;
    s->d.sslots = slots;
    s->ham_kernel = 4;
    return IRL_OK;
}

}  // namespace

extern "C" {

int irl_system_store_hamiltonian(irl_system *s, size_t max_bytes, size_t *bytes_needed, void *stream)
{
    if (!s) return set_err(nullptr, IRL_EINVAL, "system is NULL");
    const int64_t ns = s->ns;
    if (s->ham_kernel == 4) {
        if (bytes_needed)
            *bytes_needed = s->d.scb ? sliced_bytes(s->d.scb, ns, s->d.sslots)
                                     : (size_t)s->d.hcb * (ns + 1) * 8 + (size_t)s->d.hnnz * 12;
        return IRL_OK;
    }
    if (!(s->sys_flags & IRL_SYS_STORE_BLOCKS) && ((ns + ((int64_t)1 << kSliceLog) - 1) >> kSliceLog) <= kMaxSlices)
        return store_sliced(s, max_bytes, bytes_needed, (hipStream_t)stream);
    // column blocks: slices of w of about kColSliceBytes, a power of two rows wide
    int hcs = 0;
    while (hcs < 40 && ((int64_t)8 << hcs) < kColSliceBytes) ++hcs;
    while (((ns + ((int64_t)1 << hcs) - 1) >> hcs) > kMaxColBlocks) ++hcs;
    const int hcb = (int)((ns + ((int64_t)1 << hcs) - 1) >> hcs);
    hipStream_t st = (hipStream_t)stream;
    int32_t *dcount = nullptr;
    CK(s, hipMalloc((void **)&dcount, (size_t)hcb * ns * 4));
    std::vector<int32_t> count((size_t)hcb * ns);
    s->d.hcb = hcb;               // read by the count and fill passes
    s->d.hcs = hcs;
    hipError_t e = launch_ham_count(s, dcount, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(count.data(), dcount, (size_t)hcb * ns * 4, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    (void)hipFree(dcount);
    auto unset = [&]() {
        s->d.hcb = 0;
        s->d.hcs = 0;
    };
    if (e != hipSuccess) {
        unset();
        return set_err(s, IRL_EDEVICE, std::string("row counts: ") + hipGetErrorString(e));
    }
    // block-major offsets: all rows of block 0, then of block 1, ...
    std::vector<int64_t> ptr((size_t)hcb * (ns + 1));
    int64_t nnz = 0;
    for (int b = 0; b < hcb; ++b) {
        int64_t *pb = ptr.data() + (size_t)b * (ns + 1);
        const int32_t *cb = count.data() + (size_t)b * ns;
        pb[0] = nnz;
        for (int64_t r = 0; r < ns; ++r) pb[r + 1] = pb[r] + cb[r];
        nnz = pb[ns];
    }
    const size_t bytes = (size_t)hcb * (ns + 1) * 8 + (size_t)nnz * 12;
    if (bytes_needed) *bytes_needed = bytes;
    if (bytes > max_bytes) {
        unset();
        return set_err(s, IRL_ENOMEM, "stored rows need " + std::to_string(bytes) +
                                          " bytes, more than max_bytes = " + std::to_string(max_bytes));
    }
    int rc;
    const size_t bytes_before = s->dev_bytes;
    auto release = [&]() {
        s->dev_bytes = bytes_before;
        for (void *p : {(void *)s->d.hptr, (void *)s->d.hcol, (void *)s->d.hval})
            if (p) (void)hipFree(p);
        s->d.hptr = nullptr;
        s->d.hcol = nullptr;
        s->d.hval = nullptr;
        unset();
    };
    if ((rc = dev_alloc(s, &s->d.hptr, (size_t)hcb * (ns + 1))) != IRL_OK ||
        (rc = dev_alloc(s, &s->d.hcol, (size_t)nnz)) != IRL_OK ||
        (rc = dev_alloc(s, &s->d.hval, (size_t)nnz)) != IRL_OK) {
        release();
        return rc;
    }
    e = hipMemcpyAsync(s->d.hptr, ptr.data(), ptr.size() * 8, hipMemcpyHostToDevice, st);
    // targets start at row 0, so a slot the fill did not reach still gathers in bounds
    if (e == hipSuccess) e = hipMemsetAsync(s->d.hcol, 0, (size_t)std::max<int64_t>(nnz, 1) * 4, st);
    if (e == hipSuccess) e = launch_ham_fill(s, s->d.hptr, s->d.hcol, s->d.hval, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        release();
        return set_err(s, IRL_EDEVICE, std::string("stored rows: ") + hipGetErrorString(e));
    }
    s->d.hnnz = nnz;
    s->ham_kernel = 4;
    return IRL_OK;
}

int irl_system_info_get(const irl_system *s, irl_system_info *o)
{
    if (!s || !o) return IRL_EINVAL;
    o->n_dets = s->ns;
    o->n_orb = s->n;
    o->n_alpha = s->na;
    o->n_beta = s->nb;
    o->full_space = s->full ? 1 : 0;
    o->n_alpha_strings = s->full ? s->nA : -1;
    o->n_beta_strings = s->full ? s->nB : -1;
    const int va = s->n - s->na, vb = s->n - s->nb;
    o->max_connections = (int64_t)s->na * va + (int64_t)s->nb * vb +
                         binom_host(s->na, 2) * binom_host(va, 2) + binom_host(s->nb, 2) * binom_host(vb, 2) +
                         (int64_t)s->na * va * s->nb * vb;
    o->device_bytes = s->dev_bytes;
    o->ham_kernel = s->ham_kernel;
    o->stored_col_blocks = s->ham_kernel == 4 ? (s->d.scb ? s->d.scb : s->d.hcb) : 0;
    o->stored_elements = s->ham_kernel == 4 ? s->d.hnnz : 0;
    return IRL_OK;
}

int irl_workspace_query(const irl_system *s, int64_t ncols, uint32_t ws_flags, size_t *bytes)
{
    if (!s || !bytes || ncols < 2 || !(ws_flags & (IRL_WS_FP64 | IRL_WS_FP32 | IRL_WS_FACTORED)) ||
        (ws_flags & ~(uint32_t)(IRL_WS_FP64 | IRL_WS_FP32 | IRL_WS_BLOCK | IRL_WS_FACTORED | IRL_WS_SAMPLED)))
        return IRL_EINVAL;
    const WsLayout L = make_layout(s->ns, ncols, ws_flags, 2 * s->n, s->full ? s->nA : 0, s->full ? s->nB : 0);
    if ((ws_flags & IRL_WS_FACTORED) && L.hfac < 1) return IRL_EINVAL;
    *bytes = L.total;
    return IRL_OK;
}

int irl_nqs_evaluate(irl_system *s, const irl_nqs_desc *nqs, void *ws, size_t ws_bytes,
                     uint32_t ws_flags, irl_eval_out *out, void *stream)
{
    if (!s) return IRL_EINVAL;
    if (!nqs || !nqs->theta) return set_err(s, IRL_EINVAL, "network descriptor or theta is NULL");
    if (nqs->V != 2 * s->n) return set_err(s, IRL_EINVAL, "V must equal 2 * n_orb");
    if (nqs->H < 1 || nqs->H > 1024) return set_err(s, IRL_EINVAL, "H must be in [1, 1024]");
    if (!(ws_flags & (IRL_WS_FP64 | IRL_WS_FP32 | IRL_WS_FACTORED)))
        return set_err(s, IRL_EINVAL, "ws_flags names no D~ copy and no factored Jacobian");
    if ((ws_flags & IRL_WS_FACTORED) && nqs->V > 64) return set_err(s, IRL_EINVAL, "the factored Jacobian needs V <= 64");
    hipStream_t st = (hipStream_t)stream;
    const int64_t P = (int64_t)nqs->V * nqs->H + nqs->H + nqs->V;
    WsLayout L = make_layout(s->ns, P + 1, ws_flags, nqs->V, s->full ? s->nA : 0, s->full ? s->nB : 0);
    int rc = check_ws(s, ws, ws_bytes, L);
    if (rc) return rc;
    s->ws_valid = false;
    s->vmc = false;
    s->vmc_rows = 0;
    TIMED(s, IRL_STAT_DTILDE_BUILD, st, launch_nqs_dtilde(s, nqs->V, nqs->H, nqs->theta, L, ws, st));
    rc = energy_and_gradient(s, ws, L, st, nqs);
    if (rc) return rc;
    s->ws = ws;
    s->lay = L;
    s->ws_valid = true;
    s->ws_has64 = (ws_flags & (IRL_WS_FP64 | IRL_WS_FACTORED)) != 0;
    s->ws_has32 = (ws_flags & IRL_WS_FP32) != 0;
    if (out) {
        out->Z = s->Z;
        out->E = s->E_el + s->e_core;
        if (out->grad) {
            CK(s, hipMemcpyAsync(out->grad, ws_ptr<double>(ws, L.off_grad) + 1, P * 8,
                                 hipMemcpyDeviceToDevice, st));
            CK(s, hipStreamSynchronize(st));
        }
    }
    return IRL_OK;
}

int irl_adam_step(irl_system *s, const irl_nqs_desc *nqs, void *ws, size_t ws_bytes, uint32_t ws_flags,
                  const irl_adam_opts *o, double *m, double *v, int64_t t, irl_eval_out *out, void *stream)
{
    if (!s) return IRL_EINVAL;
    if (!o || !m || !v || t < 1) return set_err(s, IRL_EINVAL, "Adam options, moments or step count invalid");
    if (!(o->lr >= 0.0) || !(o->beta1 >= 0.0 && o->beta1 < 1.0) || !(o->beta2 >= 0.0 && o->beta2 < 1.0) ||
        !(o->eps > 0.0) || !std::isfinite(o->lr) || !std::isfinite(o->eps))
        return set_err(s, IRL_EINVAL, "Adam step sizes out of range");
    irl_eval_out ev{0, 0, out ? out->grad : nullptr};
    int rc = irl_nqs_evaluate(s, nqs, ws, ws_bytes, ws_flags, &ev, stream);
    if (rc) return rc;
    const int64_t P = (int64_t)nqs->V * nqs->H + nqs->H + nqs->V;
    hipStream_t st = (hipStream_t)stream;
    CK(s, launch_adam(nqs->theta, ws_ptr<double>(ws, s->lay.off_grad) + 1, m, v, P, o->lr, o->beta1, o->beta2,
                      o->eps, t, st));
    if (out) {
        out->Z = ev.Z;
        out->E = ev.E;
    }
    return IRL_OK;
}

int irl_vmc_sample(irl_system *s, void *ws, size_t ws_bytes, const double *u, int64_t n_samples,
                   int64_t *rows, double *grad_out, irl_vmc_out *out, void *stream)
{
    if (!s) return IRL_EINVAL;
    if (!s->ws_valid || s->ws != ws) return set_err(s, IRL_ESTATE, "workspace holds no evaluation for this system");
    const WsLayout L = s->lay;
    if (ws_bytes < L.total) return set_err(s, IRL_ENOMEM, "workspace too small");
    if (!u || n_samples < 1 || n_samples > 0x7fffffffLL)
        return set_err(s, IRL_EINVAL, "u is NULL or n_samples is outside [1, 2^31 - 1]");
    if (!s->ws_has64) return set_err(s, IRL_EINVAL, "the sampled gradient needs an FP64 D~ copy or the factored Jacobian");
    if ((vmc_scan_chunks(L.ns) + 1) * 8 > (int64_t)kStreamBlocks * 2 * L.ldv * 8)
        return set_err(s, IRL_EINVAL, "determinant set too large for the sampling scan");
    hipStream_t st = (hipStream_t)stream;
    if (!s->vmc) s->E_exact = s->E_el;
    const int k = 61 - std::ilogb(s->Z);
    double *dout = ws_ptr<double>(ws, L.off_r);
    s->vmc = false;
    s->vmc_rows = 0;
    TIMED(s, IRL_STAT_VMC, st, launch_vmc_sample(L, ws, u, n_samples, k, s->Z, rows, dout, st));
    const bool gather = (L.flags & IRL_WS_SAMPLED) && (L.flags & IRL_WS_FACTORED) && L.hfac > 0;
    if (gather) TIMED(s, IRL_STAT_VMC, st, launch_vmc_gather(L, ws, s->d.keys, L.hfac, st));
    double h[3];
    CK(s, hipMemcpyAsync(h, dout, sizeof(h), hipMemcpyDeviceToHost, st));
    CK(s, hipStreamSynchronize(st));
    int rc = stats_fold(s);
    if (rc) return rc;
    if (!std::isfinite(h[0])) {
        s->ws_valid = false;   // the device energy is no longer the evaluated one
        return set_err(s, IRL_EINVAL, "the sampled energy is not finite");
    }
    const int64_t nu = (int64_t)h[1];
    // sampled gradient F = (2 / Z) D~^T (q (H psi - E psi)), over the drawn rows when they
    // are gathered, else over every row from the right-hand side in the w region
    double *y = ws_ptr<double>(ws, L.off_w);
    double *grad = ws_ptr<double>(ws, L.off_grad);
    WsScalars *sc = ws_ptr<WsScalars>(ws, L.off_scal);
    int nblk = 1;
    if (gather) {
        TIMED(s, IRL_STAT_VMC, st, launch_vmc_rhs_rows(L, ws, nu, y, st));
        const FacRows R{ws_ptr<uint64_t>(ws, L.off_ckeys), nu, ws_ptr<double>(ws, L.off_cpsi),
                        ws_ptr<double>(ws, L.off_cfac)};
        nblk = fac_row_blocks_n(s, nu, L.hfac);
        TIMED(s, IRL_STAT_ENERGY, st, launch_fac_vjp_rows(s, L, ws, R, y, nullptr, nullptr, 1, nblk, st));
    } else if (L.flags & IRL_WS_FACTORED) {
        nblk = fac_vjp_blocks(s, L);
        TIMED(s, IRL_STAT_ENERGY, st, launch_fac_vjp(s, L, ws, y, nullptr, nullptr, 1, nblk, st));
    } else {
        TIMED(s, IRL_STAT_GEMV_T, st, launch_gemv_t2(L, ws, IRL_FP64, y, y, nullptr, nullptr, &nblk, st));
    }
    TIMED(s, IRL_STAT_REDUCE, st, launch_t2_reduce(L, ws, nblk, nullptr, grad, L.ncols, 2.0, &sc->Z, st));
    if (grad_out) CK(s, hipMemcpyAsync(grad_out, grad + 1, (L.ncols - 1) * 8, hipMemcpyDeviceToDevice, st));
    s->E_el = h[0];
    s->vmc = true;
    s->vmc_rows = gather ? (int64_t)h[1] : 0;
    if (out) {
        out->E_sampled = h[0] + s->e_core;
        out->E_exact = s->E_exact + s->e_core;
        out->E_loc_var = h[2];
        out->n_unique = (int64_t)h[1];
        out->n_samples = n_samples;
    }
    return IRL_OK;
}

int irl_dtilde_set(irl_system *s, const void *D, int64_t ld, int64_t ncols, int32_t dtype,
                   void *ws, size_t ws_bytes, uint32_t ws_flags, void *stream)
{
    if (!s) return IRL_EINVAL;
    if (!D || ncols < 2 || ld < ncols || (dtype != IRL_FP64 && dtype != IRL_FP32))
        return set_err(s, IRL_EINVAL, "bad D~ arguments");
    if (!(ws_flags & (IRL_WS_FP64 | IRL_WS_FP32))) return set_err(s, IRL_EINVAL, "ws_flags names no D~ copy");
    if (ws_flags & IRL_WS_FACTORED) return set_err(s, IRL_EINVAL, "a caller-set D~ has no factored form");
    hipStream_t st = (hipStream_t)stream;
    WsLayout L = make_layout(s->ns, ncols, ws_flags, 2 * s->n, s->full ? s->nA : 0, s->full ? s->nB : 0);
    int rc = check_ws(s, ws, ws_bytes, L);
    if (rc) return rc;
    s->ws_valid = false;
    s->vmc = false;
    s->vmc_rows = 0;
    TIMED(s, IRL_STAT_DTILDE_BUILD, st, launch_dtilde_import(D, ld, ncols, dtype, L, ws, st));
    rc = energy_and_gradient(s, ws, L, st);
    if (rc) return rc;
    s->ws = ws;
    s->lay = L;
    s->ws_valid = true;
    s->ws_has64 = (ws_flags & IRL_WS_FP64) != 0;
    s->ws_has32 = (ws_flags & IRL_WS_FP32) != 0;
    return IRL_OK;
}

int irl_apply_lm_operator(irl_system *s, void *ws, size_t ws_bytes, const double *v, double *yH,
                          double *yS, int32_t precision, void *stream)
{
    if (!s) return IRL_EINVAL;
    if (!s->ws_valid || ws != s->ws) return set_err(s, IRL_ESTATE, "workspace holds no evaluation for this system");
    if (ws_bytes < s->lay.total) return set_err(s, IRL_ENOMEM, "workspace too small");
    if (!v || !yH || !yS) return set_err(s, IRL_EINVAL, "NULL vector");
    int rc = check_prec(s, precision);
    if (rc) return rc;
    return apply_internal(s, ws, s->lay, v, yH, yS, precision, (hipStream_t)stream);
}

int irl_apply_lm_operator_block(irl_system *s, void *ws, size_t ws_bytes, const double *V, int64_t ldv_in,
                                int32_t nb, double *YH, double *YS, int64_t ldy, int32_t precision, void *stream)
{
    if (!s) return IRL_EINVAL;
    if (!s->ws_valid || s->ws != ws) return set_err(s, IRL_ESTATE, "workspace holds no evaluation");
    const WsLayout &L = s->lay;
    if (!(L.flags & IRL_WS_BLOCK)) return set_err(s, IRL_EINVAL, "multi-vector applies need IRL_WS_BLOCK");
    if (ws_bytes < L.total) return set_err(s, IRL_ENOMEM, "workspace too small");
    if (nb < 1 || nb > kMaxBlock) return set_err(s, IRL_EINVAL, "nb must be in [1, 8]");
    if (!V || !YH || !YS || ldv_in < L.ncols || ldy < L.ncols) return set_err(s, IRL_EINVAL, "bad vector arguments");
    int rc = check_prec(s, precision);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    return apply_block_internal(s, ws, L, V, ldv_in, nb, YH, YS, ldy, precision, st);
}

int irl_apply_hamiltonian(irl_system *s, const double *w, double *u, void *stream)
{
    if (!s || !w || !u) return IRL_EINVAL;
    CK(s, launch_ham_apply(s, w, u, (hipStream_t)stream));
    return IRL_OK;
}

int irl_step(irl_system *s, irl_nqs_desc *nqs, const irl_solver_opts *opts, void *ws,
             size_t ws_bytes, uint32_t ws_flags, double *dtheta, double *ritz, irl_step_result *r,
             void *stream)
{
    if (!s) return IRL_EINVAL;
    irl_solver_opts o;
    if (opts)
        o = *opts;
    else
        irl_solver_opts_default(&o);
    if (o.m < 2 || o.m > kMaxKrylov || o.k_keep < 1 || o.k_keep >= o.m || !(o.tol > 0.0) ||
        o.max_restarts < 0 || (o.mode != IRL_MODE_A && o.mode != IRL_MODE_P && o.mode != IRL_MODE_C) ||
        o.block < 0 || o.block > kMaxBlock)
        return set_err(s, IRL_EINVAL, "bad solver options");
    if (o.mode == IRL_MODE_C && (o.precision != IRL_FP64 || o.block > 1))
        return set_err(s, IRL_EINVAL, "the connected basis (mode C) needs an FP64 single-vector solve");
    if (o.mode == IRL_MODE_C && s->vmc && !(nqs && !(o.flags & IRL_STEP_WS_CURRENT)))
        return set_err(s, IRL_EINVAL, "the connected basis (mode C) is not defined on sampled estimators");
    hipStream_t st = (hipStream_t)stream;
    irl_step_result res;
    std::memset(&res, 0, sizeof(res));
    res.E_after = std::numeric_limits<double>::quiet_NaN();
    double t0 = now_ms();
    int rc;
    if (nqs && !(o.flags & IRL_STEP_WS_CURRENT)) {
        irl_eval_out ev{0, 0, nullptr};
        rc = irl_nqs_evaluate(s, nqs, ws, ws_bytes, ws_flags, &ev, stream);
        if (rc) return rc;
    } else if (!s->ws_valid || s->ws != ws) {
        return set_err(s, IRL_ESTATE, "workspace holds no evaluation for this system");
    }
    if (nqs) {
        const int64_t P = (int64_t)nqs->V * nqs->H + nqs->H + nqs->V;
        if (P + 1 != s->lay.ncols) return set_err(s, IRL_EINVAL, "network size does not match the workspace");
    }
    rc = check_prec(s, o.precision);
    if (rc) return rc;
    const WsLayout L = s->lay;
    res.E_before = s->E_el + s->e_core;
    double t1 = now_ms();
    res.ms_eval = t1 - t0;

    if (o.mode == IRL_MODE_C) {
        rc = connected_sigma(s, ws, L, st);
        if (rc) return rc;
    }

    // ---- implicitly restarted Lanczos ----
    SolveOut so;
    // warm start: the copy of the last converged Ritz vector, kept in its own
    // region because the evaluation at the start of a step reuses y
    const double *start = nullptr;
    if ((o.flags & IRL_STEP_WARM_START) && o.block <= 1 && s->warm_ws == ws && s->warm_ncols == L.ncols &&
        s->warm_off == L.off_warm && s->warm_mode == o.mode)
        start = ws_ptr<double>(ws, L.off_warm);
    s->warm_ws = nullptr;
    rc = o.block > 1 ? irl_solve_block(s, ws, L, o, o.precision, so, st)
                     : irl_solve(s, ws, L, o, o.precision, start, so, st);
    if (rc) return rc;
    const int n_apply_lo = o.precision == IRL_FP32 ? so.n_apply : 0;
    if (o.precision == IRL_FP32 && s->ws_has64 && !(o.flags & IRL_STEP_NO_POLISH)) {
        // FP64 polish from the reduced-precision Ritz vector
        SolveOut sp;
        rc = irl_solve(s, ws, L, o, IRL_FP64, ws_ptr<double>(ws, L.off_y), sp, st);
        if (rc) return rc;
        sp.n_apply += so.n_apply;
        sp.n_restart += so.n_restart;
        sp.n_graph += so.n_graph;
        so = sp;
    }
    double *y = ws_ptr<double>(ws, L.off_y);
    if (o.block <= 1 && so.converged) {
        CK(s, hipMemcpyAsync(ws_ptr<double>(ws, L.off_warm), y, L.ldv * 8, hipMemcpyDeviceToDevice, st));
        s->warm_ws = ws;
        s->warm_ncols = L.ncols;
        s->warm_off = L.off_warm;
        s->warm_mode = o.mode;
    }
    res.lambda_min = so.lam;
    res.residual_est = so.resid_est;
    res.residual_explicit = so.resid_explicit;
    res.gap = so.gap;
    res.norm_T = so.normT;
    res.c0 = so.c0;
    res.n_apply = so.n_apply;
    res.n_restart = so.n_restart;
    res.converged = so.converged;
    res.tol_used = so.tol_used;
    res.n_apply_lo = n_apply_lo;
    res.n_graph_cycles = so.n_graph;
    const bool converged = so.converged != 0;
    if (o.mode == IRL_MODE_C) {
        // coefficient of psi in the connected linearised wavefunction
        CK(s, launch_connected_c0(L, ws, y, st));
        rc = read_scalars(s, ws, L, st);
        if (rc) return rc;
        res.c0 = s->host_scal->c0;
    }
    if (ritz) {
        if (o.mode != IRL_MODE_P)
            CK(s, hipMemcpyAsync(ritz, y, L.ncols * 8, hipMemcpyDeviceToDevice, st));
        else
            CK(s, hipMemcpyAsync(ritz, y + 1, (L.ncols - 1) * 8, hipMemcpyDeviceToDevice, st));
    }
    double t2 = now_ms();
    res.ms_solve = t2 - t1;
    int status = converged ? IRL_OK : IRL_ENOTCONV;
    if (o.mode != IRL_MODE_P) {
        if (!(std::fabs(res.c0) >= 1e-8)) {
            status = IRL_ESTEP;
        } else {
            const bool upd = nqs && !(o.flags & IRL_STEP_NO_UPDATE);
            CK(s, launch_update(L, ws, y, dtheta, upd ? nqs->theta : nullptr, L.ncols - 1, o.mode, st));
            if (upd && !(o.flags & IRL_STEP_NO_EVAL_AFTER)) {
                irl_eval_out ev{0, 0, nullptr};
                rc = irl_nqs_evaluate(s, nqs, ws, ws_bytes, ws_flags, &ev, stream);
                if (rc) return rc;
                res.E_after = ev.E;
            }
        }
    }
    CK(s, hipStreamSynchronize(st));
    res.ms_after = now_ms() - t2;
    if (r) *r = res;
    return status;
}

int irl_stats_enable(irl_system *s, int32_t on)
{
    if (!s) return IRL_EINVAL;
    if (s->stats_on) {
        int rc = stats_fold(s);
        if (rc) return rc;
    }
    s->stats_on = on != 0;
    s->ev_open = false;
    s->ev_used = 0;
    for (int k = 0; k < IRL_STAT_KINDS; ++k) {
        s->stat_ms[k] = 0.0;
        s->stat_cnt[k] = 0;
    }
    return IRL_OK;
}

int irl_stats_select(irl_system *s, uint32_t kinds)
{
    if (!s) return IRL_EINVAL;
    if (kinds >> IRL_STAT_KINDS) return set_err(s, IRL_EINVAL, "kinds names a bit beyond the last irl_stat_kind");
    s->stat_mask = kinds;
    return IRL_OK;
}

int irl_tune_set(irl_system *s, int32_t knob, int32_t value)
{
    if (!s) return IRL_EINVAL;
    if (value < 0) return set_err(s, IRL_EINVAL, "tuning value must be 0 (default) or positive");
    switch (knob) {
    case IRL_TUNE_LUT_BLOCKS:
        if (value > 65536) return set_err(s, IRL_EINVAL, "IRL_TUNE_LUT_BLOCKS above 65536");
        s->tune_lut_blocks = value;
        return IRL_OK;
    case IRL_TUNE_PULL_BLOCKS:
        if (value > (1 << 20)) return set_err(s, IRL_EINVAL, "IRL_TUNE_PULL_BLOCKS above 2^20");
        s->tune_pull_blocks = value;
        return IRL_OK;
    case IRL_TUNE_PULL_WAVES:
        if (value != 0 && value != 1 && value != 2 && value != 4)
            return set_err(s, IRL_EINVAL, "IRL_TUNE_PULL_WAVES must be 0, 1, 2 or 4");
        s->tune_pull_waves = value;
        return IRL_OK;
    default:
        return set_err(s, IRL_EINVAL, "unknown tuning knob");
    }
}

int irl_tune_get(irl_system *s, int32_t knob, int32_t hidden, int32_t *value, int32_t *applies)
{
    if (!s || !value || !applies) return IRL_EINVAL;
    switch (knob) {
    case IRL_TUNE_LUT_BLOCKS:
        if (hidden < 1) return set_err(s, IRL_EINVAL, "hidden width must be positive");
        *value = s->tune_lut_blocks;
        *applies = irl::fac_jvp_uses_lut(s, s->ns, hidden);
        return IRL_OK;
    case IRL_TUNE_PULL_BLOCKS:
    case IRL_TUNE_PULL_WAVES:
        *value = knob == IRL_TUNE_PULL_BLOCKS ? s->tune_pull_blocks : s->tune_pull_waves;
        *applies = (s->ham_kernel == 0 || s->ham_kernel == 1 || s->ham_kernel == 3) ? 1 : 0;
        return IRL_OK;
    default:
        return set_err(s, IRL_EINVAL, "unknown tuning knob");
    }
}

int irl_stats_get(irl_system *s, double *ms, int64_t *count, void *stream)
{
    if (!s) return IRL_EINVAL;
    CK(s, hipStreamSynchronize((hipStream_t)stream));
    int rc = stats_fold(s);
    if (rc) return rc;
    for (int k = 0; k < IRL_STAT_KINDS; ++k) {
        if (ms) ms[k] = s->stat_ms[k];
        if (count) count[k] = s->stat_cnt[k];
    }
    return IRL_OK;
}

int irl_debug_keys(const irl_system *s, uint64_t *out)
{
    if (!s || !out) return IRL_EINVAL;
    if (hipMemcpy(out, s->d.keys, (size_t)s->ns * 8, hipMemcpyDeviceToHost) != hipSuccess) return IRL_EDEVICE;
    return IRL_OK;
}

int irl_debug_diagonal(const irl_system *s, double *out)
{
    if (!s || !out) return IRL_EINVAL;
    if (hipMemcpy(out, s->d.diag, (size_t)s->ns * 8, hipMemcpyDeviceToHost) != hipSuccess) return IRL_EDEVICE;
    return IRL_OK;
}

int irl_debug_lookup(const irl_system *cs, const uint64_t *keys, int64_t n, int32_t *rows)
{
    irl_system *s = const_cast<irl_system *>(cs);
    if (!s || n < 0 || (n > 0 && (!keys || !rows))) return IRL_EINVAL;
    if (n == 0) return IRL_OK;
    uint64_t *dq = nullptr;
    int32_t *dr = nullptr;
    if (hipMalloc((void **)&dq, n * 8) != hipSuccess) return IRL_ENOMEM;
    if (hipMalloc((void **)&dr, n * 4) != hipSuccess) { (void)hipFree(dq); return IRL_ENOMEM; }
    int rc = IRL_OK;
    if (hipMemcpy(dq, keys, n * 8, hipMemcpyHostToDevice) != hipSuccess ||
        launch_lookup_any(s, dq, n, dr, nullptr) != hipSuccess ||
        hipMemcpy(rows, dr, n * 4, hipMemcpyDeviceToHost) != hipSuccess)
        rc = IRL_EDEVICE;
    (void)hipFree(dq);
    (void)hipFree(dr);
    return rc;
}

int irl_lookup_noalloc(const irl_system *cs, const uint64_t *keys, int64_t n, int32_t *rows, void *stream)
{
    irl_system *s = const_cast<irl_system *>(cs);
    if (!s) return IRL_EINVAL;
    if (n < 0 || (n > 0 && (!keys || !rows))) return set_err(s, IRL_EINVAL, "bad key or row arrays");
    if (n > kNoAllocMaxKeys)
        return set_err(s, IRL_EINVAL, "irl_lookup_noalloc takes at most 262144 keys per call");
    if (n == 0) return IRL_OK;
    unsigned char *base = static_cast<unsigned char *>(noalloc_scratch(s->device));
    if (!base) return set_err(s, IRL_ESTATE, "fixed scratch not set up on this device");
    uint64_t *dq = reinterpret_cast<uint64_t *>(base);
    int32_t *dr = reinterpret_cast<int32_t *>(base + (size_t)kNoAllocMaxKeys * 8);
    hipStream_t st = (hipStream_t)stream;
    CK(s, hipMemcpyAsync(dq, keys, (size_t)n * 8, hipMemcpyHostToDevice, st));
    CK(s, launch_lookup_any(s, dq, n, dr, st));
    CK(s, hipMemcpyAsync(rows, dr, (size_t)n * 4, hipMemcpyDeviceToHost, st));
    CK(s, hipStreamSynchronize(st));
    return IRL_OK;
}

int irl_debug_excitations(const irl_system *cs, int64_t row, int32_t *target, int8_t *sign,
                          uint8_t *kind, double *hval, int64_t cap, int64_t *count)
{
    irl_system *s = const_cast<irl_system *>(cs);
    if (!s || row < 0 || row >= s->ns || !count || cap < 0) return IRL_EINVAL;
    const int64_t maxc = 4096 + 16 * 16 * 16 * 16;
    int32_t *dt = nullptr, *dc = nullptr;
    int8_t *ds = nullptr;
    uint8_t *dk = nullptr;
    double *dv = nullptr;
    int rc = IRL_OK;
    if (hipMalloc((void **)&dt, maxc * 4) != hipSuccess || hipMalloc((void **)&ds, maxc) != hipSuccess ||
        hipMalloc((void **)&dk, maxc) != hipSuccess || hipMalloc((void **)&dv, maxc * 8) != hipSuccess ||
        hipMalloc((void **)&dc, 4) != hipSuccess) {
        rc = IRL_ENOMEM;
    } else if (launch_ham_row_list(s, row, dt, ds, dk, dv, dc, (int)maxc, nullptr) != hipSuccess) {
        rc = IRL_EDEVICE;
    } else {
        int32_t c = 0;
        if (hipMemcpy(&c, dc, 4, hipMemcpyDeviceToHost) != hipSuccess) {
            rc = IRL_EDEVICE;
        } else if (c > maxc) {
            rc = IRL_EINVAL;
        } else {
            std::vector<int32_t> t(c);
            std::vector<int8_t> sg(c);
            std::vector<uint8_t> kd(c);
            std::vector<double> v(c);
            if (c && (hipMemcpy(t.data(), dt, c * 4, hipMemcpyDeviceToHost) != hipSuccess ||
                      hipMemcpy(sg.data(), ds, c, hipMemcpyDeviceToHost) != hipSuccess ||
                      hipMemcpy(kd.data(), dk, c, hipMemcpyDeviceToHost) != hipSuccess ||
                      hipMemcpy(v.data(), dv, c * 8, hipMemcpyDeviceToHost) != hipSuccess)) {
                rc = IRL_EDEVICE;
            } else {
                std::vector<int32_t> idx(c);
                for (int32_t i = 0; i < c; ++i) idx[i] = i;
                std::sort(idx.begin(), idx.end(), [&](int32_t a, int32_t b) { return t[a] < t[b]; });
                *count = c;
                if (c > cap) {
                    rc = IRL_EINVAL;
                } else {
                    for (int32_t i = 0; i < c; ++i) {
                        if (target) target[i] = t[idx[i]];
                        if (sign) sign[i] = sg[idx[i]];
                        if (kind) kind[i] = kd[idx[i]];
                        if (hval) hval[i] = v[idx[i]];
                    }
                }
            }
        }
    }
    if (dt) (void)hipFree(dt);
    if (ds) (void)hipFree(ds);
    if (dk) (void)hipFree(dk);
    if (dv) (void)hipFree(dv);
    if (dc) (void)hipFree(dc);
    return rc;
}

int irl_debug_jacobian(irl_system *s, void *ws, size_t ws_bytes, int64_t row0, int64_t nrows,
                       double *psi_host, void *rows_host, int32_t *kind, int64_t *ncols_out)
{
    if (!s) return IRL_EINVAL;
    if (!s->ws_valid || ws != s->ws) return set_err(s, IRL_ESTATE, "workspace holds no evaluation");
    const WsLayout &L = s->lay;
    if (ws_bytes < L.total) return set_err(s, IRL_ENOMEM, "workspace too small");
    if (row0 < 0 || nrows < 0 || row0 + nrows > L.ns) return set_err(s, IRL_EINVAL, "row range outside the set");
    CK(s, hipDeviceSynchronize());
    if (psi_host && nrows)
        CK(s, hipMemcpy(psi_host, ws_ptr<double>(ws, L.off_psi) + row0, (size_t)nrows * 8, hipMemcpyDeviceToHost));
    int32_t kd;
    int64_t nc;
    if ((L.flags & IRL_WS_FACTORED) && L.hfac > 0) {
        kd = 0;
        nc = L.hfac;
        if (rows_host && nrows)
            CK(s, hipMemcpy(rows_host, ws_ptr<double>(ws, L.off_fac) + row0 * (int64_t)L.hfac,
                            (size_t)nrows * L.hfac * 8, hipMemcpyDeviceToHost));
    } else if (L.flags & IRL_WS_FP64) {
        kd = 1;
        nc = L.ncols;
        if (rows_host && nrows)
            CK(s, hipMemcpy2D(rows_host, (size_t)L.ncols * 8, ws_ptr<double>(ws, L.off_d64) + row0 * L.ld64,
                              (size_t)L.ld64 * 8, (size_t)L.ncols * 8, (size_t)nrows, hipMemcpyDeviceToHost));
    } else {
        kd = 2;
        nc = L.ncols;
        if (rows_host && nrows)
            CK(s, hipMemcpy2D(rows_host, (size_t)L.ncols * 4, ws_ptr<float>(ws, L.off_d32) + row0 * L.ld32,
                              (size_t)L.ld32 * 4, (size_t)L.ncols * 4, (size_t)nrows, hipMemcpyDeviceToHost));
    }
    if (kind) *kind = kd;
    if (ncols_out) *ncols_out = nc;
    return IRL_OK;
}

int irl_debug_lanczos(irl_system *s, void *ws, size_t ws_bytes, const double *v1, int32_t j_end,
                      int32_t precision, int32_t mode, double *V_host, double *alpha_host,
                      double *beta_host, void *stream)
{
    if (!s) return IRL_EINVAL;
    if (!s->ws_valid || ws != s->ws) return set_err(s, IRL_ESTATE, "workspace holds no evaluation");
    if (ws_bytes < s->lay.total || !v1 || j_end < 1 || j_end > kMaxKrylov || (mode != IRL_MODE_A && mode != IRL_MODE_P))
        return set_err(s, IRL_EINVAL, "bad arguments");
    int rc = check_prec(s, precision);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    const WsLayout L = s->lay;
    double *V = ws_ptr<double>(ws, L.off_kry0);
    double *yH = ws_ptr<double>(ws, L.off_yh), *yS = ws_ptr<double>(ws, L.off_ys);
    CK(s, launch_reset_solve(L, ws, st));
    CK(s, hipMemsetAsync(V, 0, L.ldv * 8, st));
    CK(s, hipMemcpyAsync(V, v1, L.ncols * 8, hipMemcpyDeviceToDevice, st));
    const int split = (precision == IRL_FP32) ? 1 : 0;
    for (int j = 0; j < j_end; ++j) {
        rc = apply_internal(s, ws, L, V + (int64_t)j * L.ldv, yH, yS, precision, st, split);
        if (rc) return rc;
        CK(s, launch_lanczos_step(L, ws, V, ws_ptr<double>(ws, L.off_img0), j, mode, split, 12345, st));
    }
    rc = read_scalars(s, ws, L, st);
    if (rc) return rc;
    for (int j = 0; j < j_end; ++j) {
        if (alpha_host) alpha_host[j] = s->host_scal->alpha[j];
        if (beta_host) beta_host[j] = s->host_scal->beta[j];
    }
    if (V_host)
        for (int j = 0; j <= j_end; ++j)
            CK(s, hipMemcpy(V_host + (int64_t)j * L.ncols, V + (int64_t)j * L.ldv, L.ncols * 8,
                            hipMemcpyDeviceToHost));
    return IRL_OK;
}

}  // extern "C"

// ============================================================================
// Batches: independent solves stepped in lockstep with grouped kernels
// ============================================================================
struct irl_batch {
    int B = 0;
    std::vector<irl_system *> sys;
    std::vector<WsLayout> lay;
    std::vector<void *> ws;
    std::vector<size_t> ws_bytes;
    std::vector<irl_nqs_desc> nqs;
    std::vector<Member> hm;
    uint32_t ws_flags = 0;
    Member *dm = nullptr;
    // two device work-list regions (0: active set, 1: check / candidate set)
    WorkItem *ditems[2] = {nullptr, nullptr};
    size_t dcap[2] = {0, 0};
    WorkItem *hitems = nullptr;   // pinned staging
    size_t hcap = 0;
    MemberScalars *dscal = nullptr, *hscal = nullptr;
    int max_n = 0;   // largest orbital count among the members
};

namespace {

// work-list kinds: D~ v rows; H rows of enumerating members by lookup (string
// ranks, hash, beta blocks) and of stored-row members; D~ build rows, D~^T
// tiles, reductions, energy parts, one item per member
enum { LS_ROWS6, LS_ROWS4R, LS_ROWS4H, LS_ROWS4B, LS_ROWS4S, LS_ROWS5, LS_T2, LS_RED, LS_E1, LS_VEC,
       LS_KINDS };

struct ListSet {
    int region = 0;
    int off[LS_KINDS] = {0}, cnt[LS_KINDS] = {0};
    std::vector<int> product;   // members whose H apply is the solo string-product launch
    std::vector<int> members;   // the subset the lists cover
    int64_t blocks[LS_KINDS] = {0};   // H-row kinds: blocks of the launch (one per 4-row group)
    size_t lds6 = 0;   // dynamic LDS of the grouped D~ v launch
    const WorkItem *ptr(const irl_batch *b, int kind) const { return b->ditems[region] + off[kind]; }
};

int energy_parts(int64_t ns)
{
    return ns < (int64_t)kScalarParts * 256 ? (int)((ns + 255) / 256) : kScalarParts;
}

// Build the work lists of `subset` into device region `region` (synchronises
// the stream first: the pinned staging buffer is reused).
// lookup a member's enumerating H kernel uses (from its view taken at batch create)
int lookup_of(const Member &mb)
{
    return mb.ham.bidx ? kLkBlocks : (mb.ham.hkeys ? kLkHash : kLkRanks);
}

int build_lists(irl_batch *b, const std::vector<int> &subset, int region, int prec, ListSet &ls,
                hipStream_t st)
{
    irl_system *s0 = b->sys[0];
    std::vector<WorkItem> v;
    ls.region = region;
    auto rows = [&](int m, int64_t R) {
        const int64_t ns = b->hm[m].ns;
        for (int64_t r0 = 0; r0 < ns; r0 += R) v.push_back(WorkItem{m, 0, 0, 0, r0, std::min(ns, r0 + R)});
    };
    // H rows: one item per member, (m, first block, row groups of 4 rows)
    int64_t nblk = 0;
    auto row_groups = [&](int m) {
        const int64_t ng = (b->hm[m].ns + 3) / 4;
        v.push_back(WorkItem{m, (int)nblk, (int)ng, 0, 0, 0});
        nblk += ng;
    };
    ls.lds6 = 0;
    ls.product.clear();
    ls.members = subset;
    // enumerating H rows: most expensive members first, in short items, so the
    // launch does not end on a few long work items
    std::vector<int> by_cost(subset);
    auto row_cost = [&](int m) {
        const irl_system *s = b->sys[m];
        const int64_t va = s->n - s->na, vb = s->n - s->nb;
        return (int64_t)s->na * va * s->nb * vb + binom_host(s->na, 2) * binom_host((int)va, 2) +
               binom_host(s->nb, 2) * binom_host((int)vb, 2);
    };
    std::stable_sort(by_cost.begin(), by_cost.end(), [&](int x, int y) { return row_cost(x) > row_cost(y); });
    // D~ stream lists only for D~ copies (the factored products are solo launches)
    const bool dense = !(b->ws_flags & IRL_WS_FACTORED);
    for (int kind = 0; kind < LS_KINDS; ++kind) {
        ls.off[kind] = (int)v.size();
        const bool hrows = kind == LS_ROWS4R || kind == LS_ROWS4H || kind == LS_ROWS4B;
        nblk = 0;
        if (!dense && (kind == LS_ROWS6 || kind == LS_ROWS5 || kind == LS_T2 || kind == LS_RED)) {
            ls.cnt[kind] = 0;
            ls.blocks[kind] = 0;
            continue;
        }
        for (int m : (hrows ? by_cost : subset)) {
            const Member &mb = b->hm[m];
            // the stored rows a member uses are those in its view taken at batch create
            // LDS-sliced stored rows run their solo launch (as the string product does)
            const bool stored = mb.ham.hptr != nullptr;
            const bool product = (!stored && b->sys[m]->ham_kernel == 2) || mb.ham.sval != nullptr;
            switch (kind) {
            case LS_ROWS6: rows(m, 512); ls.lds6 = std::max(ls.lds6, (size_t)mb.ld * (prec == IRL_FP64 ? 8 : 4)); break;
            case LS_ROWS4R:
                if (product) ls.product.push_back(m);
                else if (!stored && lookup_of(mb) == kLkRanks) row_groups(m);
                break;
            case LS_ROWS4H: if (!stored && !product && lookup_of(mb) == kLkHash) row_groups(m); break;
            case LS_ROWS4B: if (!stored && !product && lookup_of(mb) == kLkBlocks) row_groups(m); break;
            case LS_ROWS4S: if (stored) row_groups(m); break;
            case LS_ROWS5: rows(m, 256); break;
            case LS_T2: {
                const int64_t nch = mb.ld / (prec == IRL_FP64 ? 2 : 4);
                const int ntiles = (int)((nch + 64 * kGroupedT2Chunks - 1) / (64 * kGroupedT2Chunks));
                const int nblk = mb.nblk_t2;
                const int64_t per = (mb.ns + nblk - 1) / nblk;
                for (int rb = 0; rb < nblk; ++rb)
                    for (int t = 0; t < ntiles; ++t) {
                        const int64_t r0 = (int64_t)rb * per;
                        v.push_back(WorkItem{m, t, rb, 0, std::min(r0, mb.ns), std::min(mb.ns, r0 + per)});
                    }
                break;
            }
            case LS_RED: {
                const int64_t len = 2 * mb.ld;
                for (int64_t a = 0; a < (len + 255) / 256; ++a) v.push_back(WorkItem{m, (int)a, 0, 0, 0, 0});
                break;
            }
            case LS_E1: {
                const int parts = mb.nparts_e;
                const int64_t per = (mb.ns + parts - 1) / parts;
                for (int p = 0; p < parts; ++p) {
                    const int64_t r0 = (int64_t)p * per;
                    v.push_back(WorkItem{m, p, 0, 0, std::min(r0, mb.ns), std::min(mb.ns, r0 + per)});
                }
                break;
            }
            case LS_VEC: v.push_back(WorkItem{m, 0, 0, 0, 0, 0}); break;
            }
        }
        ls.cnt[kind] = (int)v.size() - ls.off[kind];
        ls.blocks[kind] = nblk;
        // one launch covers the kind: grid size in work-items must stay below 2^32
        if (nblk > ((int64_t)1 << 24))
            return set_err(s0, IRL_EINVAL, "batch has more than 2^26 determinant rows of one kernel kind");
    }
    if (ls.lds6 > 64 * 1024) return set_err(s0, IRL_EINVAL, "batch member row longer than 8192 columns");
    CK(s0, hipStreamSynchronize(st));
    if (v.size() > b->hcap) {
        if (b->hitems) (void)hipHostFree(b->hitems);
        b->hitems = nullptr;
        b->hcap = 0;
        CK(s0, hipHostMalloc((void **)&b->hitems, v.size() * sizeof(WorkItem)));
        b->hcap = v.size();
    }
    if (v.size() > b->dcap[region]) {
        if (b->ditems[region]) (void)hipFree(b->ditems[region]);
        b->ditems[region] = nullptr;
        b->dcap[region] = 0;
        CK(s0, hipMalloc((void **)&b->ditems[region], v.size() * sizeof(WorkItem)));
        b->dcap[region] = v.size();
    }
    std::memcpy(b->hitems, v.data(), v.size() * sizeof(WorkItem));
    CK(s0, hipMemcpyAsync(b->ditems[region], b->hitems, v.size() * sizeof(WorkItem),
                          hipMemcpyHostToDevice, st));
    return IRL_OK;
}

int upload_members(irl_batch *b, hipStream_t st)
{
    CK(b->sys[0], hipStreamSynchronize(st));
    CK(b->sys[0], hipMemcpy(b->dm, b->hm.data(), b->B * sizeof(Member), hipMemcpyHostToDevice));
    return IRL_OK;
}

int gather(irl_batch *b, const ListSet &ls, hipStream_t st)
{
    irl_system *s0 = b->sys[0];
    TIMED(s0, IRL_STAT_RITZ, st, launch_lanczos_grouped(kGrpGather, b->dm, ls.ptr(b, LS_VEC), ls.cnt[LS_VEC], 0, 0, 0, 0, 0,
                                  b->dscal, st));
    CK(s0, hipMemcpyAsync(b->hscal, b->dscal, b->B * sizeof(MemberScalars), hipMemcpyDeviceToHost, st));
    CK(s0, hipStreamSynchronize(st));
    return IRL_OK;
}

int batch_apply(irl_batch *b, const ListSet &ls, int vsel, int j, int cur, int split, int prec,
                hipStream_t st)
{
    irl_system *s0 = b->sys[0];
    const bool factored = (b->ws_flags & IRL_WS_FACTORED) != 0;
    if (factored) {
        // each member's forward product is its solo launch (same kernel, same rows)
        for (int m : ls.members) {
            const Member &mb = b->hm[m];
            const double *v = vsel ? mb.y : mb.kry[cur] + (int64_t)j * mb.ld;
            TIMED(s0, IRL_STAT_GEMV, st, launch_fac_jvp(b->sys[m], b->lay[m], b->ws[m], v, split, mb.w, st));
        }
    } else {
        TIMED(s0, prec == IRL_FP64 ? IRL_STAT_GEMV : IRL_STAT_GEMV_LO, st, launch_gemv_rows_grouped(b->dm, ls.ptr(b, LS_ROWS6), ls.cnt[LS_ROWS6], prec, vsel, j, cur,
                                        split, ls.lds6, st));
    }
    for (int k : {LS_ROWS4R, LS_ROWS4H, LS_ROWS4B})
        if (ls.cnt[k])
            TIMED(s0, IRL_STAT_HAM_APPLY, st,
                  launch_ham_pull_grouped(b->dm, ls.ptr(b, k), ls.cnt[k], ls.blocks[k], 0,
                                          k == LS_ROWS4R ? kLkRanks : (k == LS_ROWS4H ? kLkHash : kLkBlocks), b->max_n, st));
    if (ls.cnt[LS_ROWS4S])
        TIMED(s0, IRL_STAT_HAM_APPLY, st, launch_ham_stored_grouped(b->dm, ls.ptr(b, LS_ROWS4S), ls.cnt[LS_ROWS4S], ls.blocks[LS_ROWS4S], 0, st));
    for (int m : ls.product) TIMED(s0, IRL_STAT_HAM_APPLY, st, launch_ham_apply(b->sys[m], b->hm[m].w, b->hm[m].u, st));
    if (factored) {
        // both backward products in one pass and the fixed-order reduction, per member
        for (int m : ls.members) {
            const WsLayout &L = b->lay[m];
            const Member &mb = b->hm[m];
            const int nb = fac_vjp_blocks(b->sys[m], L);
            TIMED(s0, IRL_STAT_GEMV_T, st, launch_fac_vjp(b->sys[m], L, b->ws[m], mb.w, mb.u, nullptr, 0, nb, st));
            TIMED(s0, IRL_STAT_REDUCE, st, launch_t2_reduce(L, b->ws[m], nb, mb.yS, mb.yH, L.ncols, 1.0, nullptr, st));
        }
        return IRL_OK;
    }
    TIMED(s0, prec == IRL_FP64 ? IRL_STAT_GEMV_T : IRL_STAT_GEMV_T_LO, st, launch_gemv_t2_grouped(b->dm, ls.ptr(b, LS_T2), ls.cnt[LS_T2], prec, 0, st));
    TIMED(s0, IRL_STAT_REDUCE, st, launch_reduce_grouped(b->dm, ls.ptr(b, LS_RED), ls.cnt[LS_RED], 0, st));
    return IRL_OK;
}

// the D~^T launches of a phase use the row blocks of the solo launch at that precision
int set_stream_precision(irl_batch *b, int prec, hipStream_t st)
{
    bool changed = false;
    for (int i = 0; i < b->B; ++i) {
        const int nb = t2_blocks(b->hm[i].ns, b->hm[i].ld, prec);
        if (nb != b->hm[i].nblk_t2) {
            b->hm[i].nblk_t2 = nb;
            changed = true;
        }
    }
    return changed ? upload_members(b, st) : IRL_OK;
}

int batch_evaluate(irl_batch *b, const std::vector<int> &subset, hipStream_t st)
{
    irl_system *s0 = b->sys[0];
    ListSet ls;
    const bool factored = (b->ws_flags & IRL_WS_FACTORED) != 0;
    const int prec = (b->ws_flags & (IRL_WS_FP64 | IRL_WS_FACTORED)) ? IRL_FP64 : IRL_FP32;
    int rc = factored ? IRL_OK : set_stream_precision(b, prec, st);
    if (rc) return rc;
    rc = build_lists(b, subset, 0, prec, ls, st);
    if (rc) return rc;
    if (factored) {
        for (int m : subset)
            TIMED(s0, IRL_STAT_DTILDE_BUILD, st, launch_fac_forward(b->sys[m], b->lay[m], b->ws[m], b->nqs[m].theta, st));
    } else {
        TIMED(s0, IRL_STAT_DTILDE_BUILD, st, launch_nqs_dtilde_grouped(b->dm, ls.ptr(b, LS_ROWS5), ls.cnt[LS_ROWS5], 0, 0, st));
    }
    for (int k : {LS_ROWS4R, LS_ROWS4H, LS_ROWS4B})
        if (ls.cnt[k])
            TIMED(s0, IRL_STAT_HAM_APPLY, st,
                  launch_ham_pull_grouped(b->dm, ls.ptr(b, k), ls.cnt[k], ls.blocks[k], 1,
                                          k == LS_ROWS4R ? kLkRanks : (k == LS_ROWS4H ? kLkHash : kLkBlocks), b->max_n, st));
    if (ls.cnt[LS_ROWS4S])
        TIMED(s0, IRL_STAT_HAM_APPLY, st, launch_ham_stored_grouped(b->dm, ls.ptr(b, LS_ROWS4S), ls.cnt[LS_ROWS4S], ls.blocks[LS_ROWS4S], 1, st));
    for (int m : ls.product) TIMED(s0, IRL_STAT_HAM_APPLY, st, launch_ham_apply(b->sys[m], b->hm[m].psi, b->hm[m].hpsi, st));
    TIMED(s0, IRL_STAT_ENERGY, st, launch_energy_grouped(b->dm, ls.ptr(b, LS_E1), ls.cnt[LS_E1], 1, st));
    TIMED(s0, IRL_STAT_ENERGY, st, launch_energy_grouped(b->dm, ls.ptr(b, LS_VEC), ls.cnt[LS_VEC], 2, st));
    if (factored) {
        // gradient: the solo backward product with c = H psi - E psi, per member
        for (int m : subset) {
            const WsLayout &L = b->lay[m];
            const Member &mb = b->hm[m];
            const int nb = fac_vjp_blocks(b->sys[m], L);
            TIMED(s0, IRL_STAT_ENERGY, st, launch_fac_vjp(b->sys[m], L, b->ws[m], mb.hpsi, nullptr, &mb.sc->E_el, 1, nb, st));
            TIMED(s0, IRL_STAT_REDUCE, st, launch_t2_reduce(L, b->ws[m], nb, nullptr, mb.grad, L.ncols, 2.0, &mb.sc->Z, st));
        }
    } else if (prec == IRL_FP64) {
        TIMED(s0, IRL_STAT_GEMV_T, st, launch_gemv_t2_grouped(b->dm, ls.ptr(b, LS_T2), ls.cnt[LS_T2], prec, 1, st));
        TIMED(s0, IRL_STAT_REDUCE, st, launch_reduce_grouped(b->dm, ls.ptr(b, LS_RED), ls.cnt[LS_RED], 1, st));
    } else {
        // no FP64 copy: each member's FP64 gradient is recomputed from its theta (solo launches)
        for (int m : subset) {
            const WsLayout &L = b->lay[m];
            const int nblk = t2_blocks(L.ns, L.ld32, IRL_FP32);
            TIMED(s0, IRL_STAT_ENERGY, st, launch_nqs_grad(b->sys[m], b->nqs[m].V, b->nqs[m].H, b->nqs[m].theta,
                                                            L, b->ws[m], nblk, st));
            TIMED(s0, IRL_STAT_REDUCE, st,
                  launch_t2_reduce(L, b->ws[m], nblk, nullptr, ws_ptr<double>(b->ws[m], L.off_grad), L.ncols,
                                   2.0, &ws_ptr<WsScalars>(b->ws[m], L.off_scal)->Z, st));
        }
    }
    rc = gather(b, ls, st);
    if (rc) return rc;
    for (int m : subset) {
        irl_system *s = b->sys[m];
        s->Z = b->hscal[m].Z;
        s->E_el = b->hscal[m].E_el;
        s->ws = b->ws[m];
        s->lay = b->lay[m];
        s->ws_valid = true;
        s->vmc = false;
        s->vmc_rows = 0;
        s->ws_has64 = (b->ws_flags & (IRL_WS_FP64 | IRL_WS_FACTORED)) != 0;
        s->ws_has32 = (b->ws_flags & IRL_WS_FP32) != 0;
        if (!(s->Z > 0.0) || !std::isfinite(s->E_el))
            return set_err(s0, IRL_EINVAL, "batch member " + std::to_string(m) + ": psi^T psi is zero or the energy is not finite");
    }
    return IRL_OK;
}

struct MemberSolve {
    double lam = 0, resid_est = 0, resid_explicit = 0, gap = 0, normT = 0, c0 = 0, tol_used = 0;
    int n_apply = 0, n_restart = 0, converged = 0, done = 0;
};

// Lockstep IRL over all members (irl_solve semantics per member).
int batch_solve(irl_batch *b, const irl_solver_opts &o, int prec, bool from_y,
                std::vector<MemberSolve> &out, hipStream_t st)
{
    irl_system *s0 = b->sys[0];
    const int B = b->B;
    int m = o.m, k = o.k_keep;
    for (int i = 0; i < B; ++i) {
        const int64_t dim = (o.mode == IRL_MODE_A) ? b->hm[i].ncols : b->hm[i].ncols - 1;
        if (dim < m) return set_err(s0, IRL_EINVAL, "batch member too small for the Krylov dimension");
    }
    const double u_op = (prec == IRL_FP64) ? 1.1102230246251565e-16 : 5.960464477539063e-08;
    const int split = (prec == IRL_FP32) ? 1 : 0;
    std::vector<int> stride(B);
    for (int i = 0; i < B; ++i) {
        const double apply_bytes = 2.0 * (double)b->hm[i].ns * (double)b->hm[i].ld * (prec == IRL_FP64 ? 8.0 : 4.0);
        stride[i] = (o.flags & IRL_STEP_FULL_CYCLES) ? 0 : (apply_bytes >= 2.56e8 ? kCheckStride : 0);
    }
    out.assign(B, MemberSolve());
    std::vector<int> active(B);
    for (int i = 0; i < B; ++i) active[i] = i;
    ListSet la, lc;
    int rc = set_stream_precision(b, prec, st);
    if (rc) return rc;
    rc = build_lists(b, active, 0, prec, la, st);
    if (rc) return rc;
    TIMED(s0, IRL_STAT_RITZ, st, launch_lanczos_grouped(kGrpReset, b->dm, la.ptr(b, LS_VEC), la.cnt[LS_VEC], 0, 0, 0, 0, 0, nullptr, st));
    TIMED(s0, IRL_STAT_RITZ, st, launch_lanczos_grouped(kGrpStart, b->dm, la.ptr(b, LS_VEC), la.cnt[LS_VEC], o.mode, from_y ? 1 : 0, 0, 0, o.seed, nullptr, st));
    int j0 = 0, cur = 0, n_restart = 0;
    // test candidates: Ritz vector of T_mc, one explicit apply, residual
    auto finalize = [&](const std::vector<int> &cand, int mc, bool accept_all) -> int {
        if (cand.empty()) return IRL_OK;
        int r2 = build_lists(b, cand, 1, prec, lc, st);
        if (r2) return r2;
        TIMED(s0, IRL_STAT_RITZ, st, launch_lanczos_grouped(kGrpRitzVector, b->dm, lc.ptr(b, LS_VEC), lc.cnt[LS_VEC], cur, mc, 0, 0, 0, nullptr, st));
        TIMED(s0, IRL_STAT_RITZ, st, launch_lanczos_grouped(kGrpResidual, b->dm, lc.ptr(b, LS_VEC), lc.cnt[LS_VEC], o.mode, 0, 0, 0, 0, nullptr, st));
        r2 = gather(b, lc, st);
        if (r2) return r2;
        std::vector<int> still;
        for (int i : cand) {
            MemberSolve &ms = out[i];
            ms.resid_explicit = std::sqrt(b->hscal[i].resid2);
            ms.c0 = b->hscal[i].c0;
            const double tol_explicit = std::max(ms.tol_used, 1024.0 * u_op * ms.normT);
            if (accept_all || ms.resid_explicit <= tol_explicit) {
                ms.converged = accept_all ? 0 : 1;
                ms.done = 1;
                ms.n_restart = n_restart;
            }
        }
        std::vector<int> na;
        for (int i : active)
            if (!out[i].done) na.push_back(i);
        if (na.size() != active.size()) {
            active.swap(na);
            if (!active.empty()) {
                int r3 = build_lists(b, active, 0, prec, la, st);
                if (r3) return r3;
            }
        }
        return IRL_OK;
    };
    auto check = [&](const std::vector<int> &who, int mt, int kk, bool end_of_cycle, std::vector<int> &cand) -> int {
        cand.clear();
        if (who.empty()) return IRL_OK;
        int r2 = build_lists(b, who, 1, prec, lc, st);
        if (r2) return r2;
        TIMED(s0, IRL_STAT_RITZ, st, launch_lanczos_grouped(kGrpRitz, b->dm, lc.ptr(b, LS_VEC), lc.cnt[LS_VEC], mt, kk, 0, 0, 0, nullptr, st));
        r2 = gather(b, lc, st);
        if (r2) return r2;
        for (int i : who) {
            const MemberScalars &hs = b->hscal[i];
            if (!std::isfinite(hs.lam)) return set_err(s0, IRL_EINVAL, "non-finite Ritz value in batch member " + std::to_string(i));
            const double tq = std::max(o.tol, 64.0 * u_op * hs.normT);
            MemberSolve &ms = out[i];
            if (end_of_cycle || hs.resid_est <= tq) {
                ms.lam = hs.lam;
                ms.resid_est = hs.resid_est;
                ms.gap = hs.gap;
                ms.normT = hs.normT;
                ms.tol_used = tq;
            }
            if (hs.resid_est <= tq) cand.push_back(i);
        }
        return IRL_OK;
    };
    std::vector<int> cand;
    while (!active.empty()) {
        bool cycle_done = true;
        for (int j = j0; j < m && !active.empty(); ++j) {
            rc = batch_apply(b, la, 0, j, cur, split, prec, st);
            if (rc) return rc;
            for (int i : active) out[i].n_apply += 1;
            TIMED(s0, IRL_STAT_LANCZOS, st, launch_lanczos_grouped(kGrpLanczos, b->dm, la.ptr(b, LS_VEC), la.cnt[LS_VEC], j, cur, o.mode, split,
                                          o.seed, nullptr, st));
            if (j + 1 < m && j + 1 >= 2 && (j + 1 - j0) % kCheckStride == 0) {
                std::vector<int> who;
                for (int i : active)
                    if (stride[i]) who.push_back(i);
                rc = check(who, j + 1, 0, false, cand);
                if (rc) return rc;
                rc = finalize(cand, j + 1, false);
                if (rc) return rc;
            }
            if (active.empty()) cycle_done = false;
        }
        if (!cycle_done || active.empty()) break;
        rc = check(active, m, k, true, cand);
        if (rc) return rc;
        rc = finalize(cand, m, false);
        if (rc) return rc;
        if (active.empty()) break;
        if (n_restart >= o.max_restarts) {
            std::vector<int> rest = active;
            rc = check(rest, m, 0, true, cand);
            if (rc) return rc;
            rc = finalize(rest, m, true);
            if (rc) return rc;
            break;
        }
        TIMED(s0, IRL_STAT_RITZ, st, launch_lanczos_grouped(kGrpRestart, b->dm, la.ptr(b, LS_VEC), la.cnt[LS_VEC], cur, m, k, o.mode,
                                      o.seed, nullptr, st));
        cur = 1 - cur;
        j0 = k;
        ++n_restart;
    }
    return IRL_OK;
}

}  // namespace

extern "C" {

int irl_batch_create(int32_t count, irl_system *const *systems, const irl_nqs_desc *nqs,
                     void *const *ws, const size_t *ws_bytes, uint32_t ws_flags, irl_batch **out)
{
    if (!out) return IRL_EINVAL;
    *out = nullptr;
    if (count < 1 || !systems || !nqs || !ws || !ws_bytes) return set_err(nullptr, IRL_EINVAL, "bad batch arguments");
    if (!(ws_flags & (IRL_WS_FP64 | IRL_WS_FP32 | IRL_WS_FACTORED)))
        return set_err(nullptr, IRL_EINVAL, "ws_flags names no D~ copy and no factored Jacobian");
    if ((ws_flags & IRL_WS_FACTORED) && (ws_flags & (IRL_WS_FP64 | IRL_WS_FP32)))
        return set_err(nullptr, IRL_EINVAL, "batch workspaces hold either D~ copies or the factored Jacobian");
    if (ws_flags & IRL_WS_SAMPLED) return set_err(nullptr, IRL_EINVAL, "batches use the exact estimators");
    irl_batch *b = new irl_batch();
    b->B = count;
    b->ws_flags = ws_flags;
    for (int i = 0; i < count; ++i) {
        irl_system *s = systems[i];
        if (!s || !nqs[i].theta) { delete b; return set_err(nullptr, IRL_EINVAL, "NULL batch member"); }
        for (int k = 0; k < i; ++k)
            if (systems[k] == s) { delete b; return set_err(nullptr, IRL_EINVAL, "a system appears twice in a batch"); }
        if (nqs[i].V != 2 * s->n || nqs[i].H < 1 || nqs[i].H > 1024) { delete b; return set_err(nullptr, IRL_EINVAL, "bad network size in batch member " + std::to_string(i)); }
        if ((ws_flags & IRL_WS_FACTORED) && nqs[i].V > 64) { delete b; return set_err(nullptr, IRL_EINVAL, "the factored Jacobian needs V <= 64"); }
        const int64_t P = (int64_t)nqs[i].V * nqs[i].H + nqs[i].H + nqs[i].V;
        WsLayout L = make_layout(s->ns, P + 1, ws_flags, nqs[i].V, s->full ? s->nA : 0, s->full ? s->nB : 0);
        if (L.ldv > 8192) { delete b; return set_err(nullptr, IRL_EINVAL, "batch members need P + 1 <= 8192"); }
        if (!ws[i] || reinterpret_cast<uintptr_t>(ws[i]) % 256 || ws_bytes[i] < L.total) { delete b; return set_err(nullptr, IRL_ENOMEM, "batch workspace missing or too small for member " + std::to_string(i)); }
        b->sys.push_back(s);
        b->max_n = std::max(b->max_n, (int)s->n);
        b->lay.push_back(L);
        b->ws.push_back(ws[i]);
        b->ws_bytes.push_back(ws_bytes[i]);
        b->nqs.push_back(nqs[i]);
        Member mb;
        std::memset(&mb, 0, sizeof(mb));
        mb.ham = ham_view(s);
        mb.D64 = (ws_flags & IRL_WS_FP64) ? ws_ptr<double>(ws[i], L.off_d64) : nullptr;
        mb.D32 = (ws_flags & IRL_WS_FP32) ? ws_ptr<float>(ws[i], L.off_d32) : nullptr;
        mb.ld = L.ldv;
        mb.ncols = L.ncols;
        mb.ns = L.ns;
        mb.psi = ws_ptr<double>(ws[i], L.off_psi);
        mb.hpsi = ws_ptr<double>(ws[i], L.off_hpsi);
        mb.w = ws_ptr<double>(ws[i], L.off_w);
        mb.u = ws_ptr<double>(ws[i], L.off_u);
        mb.grad = ws_ptr<double>(ws[i], L.off_grad);
        mb.yH = ws_ptr<double>(ws[i], L.off_yh);
        mb.yS = ws_ptr<double>(ws[i], L.off_ys);
        mb.y = ws_ptr<double>(ws[i], L.off_y);
        mb.hy = ws_ptr<double>(ws[i], L.off_hy);
        mb.img[0] = ws_ptr<double>(ws[i], L.off_img0);
        mb.img[1] = ws_ptr<double>(ws[i], L.off_img1);
        mb.r = ws_ptr<double>(ws[i], L.off_r);
        mb.part = ws_ptr<double>(ws[i], L.off_part);
        mb.part2 = ws_ptr<double>(ws[i], L.off_part2);
        mb.red = ws_ptr<double>(ws[i], L.off_red);
        mb.vconv = ws_ptr<double>(ws[i], L.off_vconv);
        mb.kry[0] = ws_ptr<double>(ws[i], L.off_kry0);
        mb.kry[1] = ws_ptr<double>(ws[i], L.off_kry1);
        mb.sc = ws_ptr<WsScalars>(ws[i], L.off_scal);
        mb.V = nqs[i].V;
        mb.H = nqs[i].H;
        mb.theta = nqs[i].theta;
        mb.dtheta = nullptr;
        mb.nblk_t2 = t2_blocks(L.ns, L.ldv, (ws_flags & IRL_WS_FP64) ? IRL_FP64 : IRL_FP32);
        mb.nparts_e = energy_parts(L.ns);
        b->hm.push_back(mb);
    }
    irl_system *s0 = b->sys[0];
    if (hipMalloc((void **)&b->dm, count * sizeof(Member)) != hipSuccess ||
        hipMalloc((void **)&b->dscal, count * sizeof(MemberScalars)) != hipSuccess ||
        hipHostMalloc((void **)&b->hscal, count * sizeof(MemberScalars)) != hipSuccess) {
        irl_batch_destroy(b);
        return set_err(s0, IRL_ENOMEM, "batch descriptors");
    }
    if (hipMemcpy(b->dm, b->hm.data(), count * sizeof(Member), hipMemcpyHostToDevice) != hipSuccess) {
        irl_batch_destroy(b);
        return set_err(s0, IRL_EDEVICE, "batch descriptor upload");
    }
    *out = b;
    return IRL_OK;
}

void irl_batch_destroy(irl_batch *b)
{
    if (!b) return;
    if (b->dm) (void)hipFree(b->dm);
    for (int r = 0; r < 2; ++r)
        if (b->ditems[r]) (void)hipFree(b->ditems[r]);
    if (b->hitems) (void)hipHostFree(b->hitems);
    if (b->dscal) (void)hipFree(b->dscal);
    if (b->hscal) (void)hipHostFree(b->hscal);
    delete b;
}

int irl_batch_step(irl_batch *b, const irl_solver_opts *opts, double *const *dtheta,
                   irl_step_result *results, int32_t *status, void *stream)
{
    if (!b) return IRL_EINVAL;
    irl_system *s0 = b->sys[0];
    irl_solver_opts o;
    if (opts)
        o = *opts;
    else
        irl_solver_opts_default(&o);
    if (o.m < 2 || o.m > kMaxKrylov || o.k_keep < 1 || o.k_keep >= o.m || !(o.tol > 0.0) ||
        o.max_restarts < 0 || (o.mode != IRL_MODE_A && o.mode != IRL_MODE_P))
        return set_err(s0, IRL_EINVAL, "bad solver options");
    if (o.block > 1) return set_err(s0, IRL_EINVAL, "batches step with single-vector Lanczos (block must be 0 or 1)");
    if ((o.precision == IRL_FP64 && !(b->ws_flags & (IRL_WS_FP64 | IRL_WS_FACTORED))) ||
        (o.precision == IRL_FP32 && !(b->ws_flags & IRL_WS_FP32)))
        return set_err(s0, IRL_ESTATE, "batch workspaces hold no D~ copy or factored Jacobian for this precision");
    hipStream_t st = (hipStream_t)stream;
    const int B = b->B;
    std::vector<int> all(B);
    for (int i = 0; i < B; ++i) all[i] = i;
    std::vector<irl_step_result> res(B);
    for (auto &r : res) {
        std::memset(&r, 0, sizeof(r));
        r.E_after = std::numeric_limits<double>::quiet_NaN();
    }
    for (int i = 0; i < B; ++i) {
        b->hm[i].theta = b->nqs[i].theta;
        b->hm[i].dtheta = nullptr;
    }
    int rc = upload_members(b, st);
    if (rc) return rc;
    const double t0 = now_ms();
    if (!(o.flags & IRL_STEP_WS_CURRENT)) {
        rc = batch_evaluate(b, all, st);
        if (rc) return rc;
    } else {
        for (int i = 0; i < B; ++i)
            if (!b->sys[i]->ws_valid || b->sys[i]->ws != b->ws[i])
                return set_err(s0, IRL_ESTATE, "batch member " + std::to_string(i) + " holds no evaluation");
    }
    for (int i = 0; i < B; ++i) res[i].E_before = b->sys[i]->E_el + b->sys[i]->e_core;
    const double t1 = now_ms();
    std::vector<MemberSolve> ms;
    rc = batch_solve(b, o, o.precision, false, ms, st);
    if (rc) return rc;
    std::vector<int> lo(B, 0);
    if (o.precision == IRL_FP32)
        for (int i = 0; i < B; ++i) lo[i] = ms[i].n_apply;
    if (o.precision == IRL_FP32 && (b->ws_flags & IRL_WS_FP64) && !(o.flags & IRL_STEP_NO_POLISH)) {
        std::vector<MemberSolve> mp;
        rc = batch_solve(b, o, IRL_FP64, true, mp, st);
        if (rc) return rc;
        for (int i = 0; i < B; ++i) {
            mp[i].n_apply += ms[i].n_apply;
            mp[i].n_restart += ms[i].n_restart;
        }
        ms.swap(mp);
    }
    const double t2 = now_ms();
    std::vector<int> upd;
    for (int i = 0; i < B; ++i) {
        irl_step_result &r = res[i];
        r.lambda_min = ms[i].lam;
        r.residual_est = ms[i].resid_est;
        r.residual_explicit = ms[i].resid_explicit;
        r.gap = ms[i].gap;
        r.norm_T = ms[i].normT;
        r.c0 = ms[i].c0;
        r.n_apply = ms[i].n_apply;
        r.n_restart = ms[i].n_restart;
        r.converged = ms[i].converged;
        r.tol_used = ms[i].tol_used;
        r.n_apply_lo = lo[i];
        int stt = ms[i].converged ? IRL_OK : IRL_ENOTCONV;
        if (o.mode == IRL_MODE_A) {
            if (!(std::fabs(r.c0) >= 1e-8))
                stt = IRL_ESTEP;
            else
                upd.push_back(i);
        }
        if (status) status[i] = stt;
    }
    if (!upd.empty()) {
        const bool move = !(o.flags & IRL_STEP_NO_UPDATE);
        for (int i : upd) {
            b->hm[i].dtheta = dtheta ? dtheta[i] : nullptr;
            b->hm[i].theta = move ? b->nqs[i].theta : nullptr;
        }
        rc = upload_members(b, st);
        if (rc) return rc;
        ListSet lu;
        rc = build_lists(b, upd, 1, o.precision, lu, st);
        if (rc) return rc;
        TIMED(s0, IRL_STAT_RITZ, st, launch_lanczos_grouped(kGrpUpdate, b->dm, lu.ptr(b, LS_VEC), lu.cnt[LS_VEC], 0, 0, 0, 0, 0, nullptr, st));
        for (int i = 0; i < B; ++i) {
            b->hm[i].theta = b->nqs[i].theta;
            b->hm[i].dtheta = nullptr;
        }
        rc = upload_members(b, st);
        if (rc) return rc;
        if (move && !(o.flags & IRL_STEP_NO_EVAL_AFTER)) {
            rc = batch_evaluate(b, upd, st);
            if (rc) return rc;
            for (int i : upd) res[i].E_after = b->sys[i]->E_el + b->sys[i]->e_core;
        }
    }
    CK(s0, hipStreamSynchronize(st));
    const double t3 = now_ms();
    for (int i = 0; i < B; ++i) {
        res[i].ms_eval = t1 - t0;
        res[i].ms_solve = t2 - t1;
        res[i].ms_after = t3 - t2;
        if (results) results[i] = res[i];
    }
    return IRL_OK;
}

}  // extern "C"
