// Lanczos recurrence, Ritz pairs and implicit restart on gfx950 (FP64).
//
// Algorithm 2 (Lanczos tridiagonal reduction) and Algorithm 1 (implicitly
// restarted Lanczos), Methods "The Standard Lanczos Process and Implicit
// Restart":
//   alpha_j = v_j^T w, w <- w - alpha_j v_j - beta_{j-1} v_{j-1},
//   beta_j = ||w||, v_{j+1} = w / beta_j;
//   T_m = tridiag(beta, alpha, beta), H V_m = V_m T_m + beta_m v_{m+1} e_m^T;
//   Ritz pairs from T_m U = U Lambda; the unwanted Ritz values are applied as
//   mu = m - k exact shifts by implicit shifted QR steps on T_m, and the
//   Lanczos factorisation is compressed to k vectors and extended again.
// Additions to the printed recurrence: two passes of classical Gram-Schmidt
// against all previous basis vectors after every step, and a breakdown
// (beta_j ~ 0) continues with a fresh random vector orthogonal to the basis.
//
// The operator seen by the Lanczos process is the centred matrix
//   H~' v = (y_H - E y_S) / Z,  (y_H, y_S) = (D~^T H D~ v, D~^T D~ v)
// (Eqs. heff and standard_evp with <psi|psi> = 1 realised by 1/Z).  Mode P
// keeps component 0 of every vector at zero, which restricts H~' to H_eff.
//
// Vector kernels run in one 1024-thread workgroup (vectors are P+1 <= ~1e5
// long); the tridiagonal eigen-solver and the QR restart run in one wavefront
// with lanes owning rows of the accumulated rotation matrix.
#include "internal.h"

namespace irl {

constexpr int kVecThreads = 1024;
constexpr int kVecWaves = kVecThreads / kWave;

__device__ __forceinline__ uint64_t splitmix64(uint64_t seed, uint64_t idx)
{
    uint64_t z = seed + (idx + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
__device__ __forceinline__ double uniform_pm1(uint64_t seed, uint64_t idx)
{
    return (double)(splitmix64(seed, idx) >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

// Block-wide sum over 1024 threads, fixed order; result broadcast to all.
__device__ double block_sum(double v, double *sh)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    __syncthreads();
    if (lane == 0) sh[wv] = v;
    __syncthreads();
    double s = 0.0;
    for (int i = 0; i < kVecWaves; ++i) s += sh[i];
    return s;
}

// h[d] = V[d] . w for d < nd (fixed order), into shared hsh[nd]
__device__ void block_dots(const double *V, int64_t ldv, int nd, const double *w, int64_t L,
                           double *sh, double *hsh)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    __syncthreads();
    for (int d = 0; d < nd; ++d) {
        double p = 0.0;
        for (int64_t i = threadIdx.x; i < L; i += kVecThreads) p += V[d * ldv + i] * w[i];
        for (int off = 32; off > 0; off >>= 1) p += __shfl_xor(p, off, kWave);
        if (lane == 0) sh[wv * (kMaxKrylov + 1) + d] = p;
    }
    __syncthreads();
    if (threadIdx.x < nd) {
        double s = 0.0;
        for (int i = 0; i < kVecWaves; ++i) s += sh[i * (kMaxKrylov + 1) + threadIdx.x];
        hsh[threadIdx.x] = s;
    }
    __syncthreads();
}

// w -= sum_d h[d] V[d]   (each element owned by one thread: no race)
__device__ void block_sub(const double *V, int64_t ldv, int nd, const double *hsh, double *w,
                          int64_t L)
{
    for (int64_t i = threadIdx.x; i < L; i += kVecThreads) {
        double x = w[i];
        for (int d = 0; d < nd; ++d) x -= hsh[d] * V[d * ldv + i];
        w[i] = x;
    }
    __syncthreads();
}

// two passes of classical Gram-Schmidt of w against V[0..nd); returns the
// accumulated coefficient of V[nd-1]
__device__ double cgs2(const double *V, int64_t ldv, int nd, double *w, int64_t L, double *sh,
                       double *hsh)
{
    double last = 0.0;
    for (int pass = 0; pass < 2; ++pass) {
        block_dots(V, ldv, nd, w, L, sh, hsh);
        if (nd > 0) last += hsh[nd - 1];
        block_sub(V, ldv, nd, hsh, w, L);
    }
    return last;
}

// random unit vector orthogonal to V[0..nd) into w (component 0 zero in mode P)
__device__ double fresh_vector(const double *V, int64_t ldv, int nd, double *w, int64_t L,
                               int64_t ncols, int mode, uint64_t seed, double *sh, double *hsh)
{
    for (int64_t i = threadIdx.x; i < L; i += kVecThreads)
        w[i] = (i < ncols && !(mode == IRL_MODE_P && i == 0)) ? uniform_pm1(seed, (uint64_t)i) : 0.0;
    __syncthreads();
    cgs2(V, ldv, nd, w, L, sh, hsh);
    double p = 0.0;
    for (int64_t i = threadIdx.x; i < L; i += kVecThreads) p += w[i] * w[i];
    double nrm = sqrt(block_sum(p, sh));
    for (int64_t i = threadIdx.x; i < L; i += kVecThreads) w[i] = nrm > 0.0 ? w[i] / nrm : 0.0;
    __syncthreads();
    return nrm;
}

// (H~' v)_i from the raw operator pair.  Plain form: (yH_i - E yS_i) / Z.  Split
// form (pair computed from (0, v[1:])): component 0 is g.v[1:] / 2 and
// components i >= 1 add g_i v_0 / 2, with g = grad[1:] in FP64.
__device__ __forceinline__ double centred_component(int64_t i, const double *yH, const double *yS,
                                                    const double *grad, double v0, double gdotv,
                                                    double Z, double E, int split)
{
    if (split) {
        if (i == 0) return 0.5 * gdotv;
        return (yH[i] - E * yS[i]) / Z + 0.5 * grad[i] * v0;
    }
    return (yH[i] - E * yS[i]) / Z;
}

// g.v[1:] over the block (only needed in split form)
__device__ double grad_dot(const double *grad, const double *v, int64_t ncols, double *sh)
{
    double p = 0.0;
    for (int64_t i = 1 + threadIdx.x; i < ncols; i += kVecThreads) p += grad[i] * v[i];
    return block_sum(p, sh);
}

__global__ __launch_bounds__(kVecThreads) void k_start_vector(double *v, int64_t ncols, int64_t ldv,
                                                             int mode, uint64_t seed)
{
    __shared__ double sh[kVecWaves * (kMaxKrylov + 1)];
    __shared__ double hsh[kMaxKrylov + 1];
    fresh_vector(nullptr, ldv, 0, v, ldv, ncols, mode, seed, sh, hsh);
}

hipError_t launch_start_vector(double *v, int64_t ncols, int64_t ldv, int mode, uint64_t seed,
                               hipStream_t st)
{
    k_start_vector<<<1, kVecThreads, 0, st>>>(v, ncols, ldv, mode, seed);
    return hipGetLastError();
}

// One Lanczos step j: w = H~' v_j from (yH, yS), recurrence, CGS2, normalise.
__device__ void lanczos_step_body(
    const double *__restrict__ yH, const double *__restrict__ yS, const double *__restrict__ grad,
    WsScalars *sc, double *V, int64_t ldv, int64_t ncols, int j, int mode, int split, uint64_t seed)
{
    __shared__ double sh[kVecWaves * (kMaxKrylov + 1)];
    __shared__ double hsh[kMaxKrylov + 1];
    const double Z = sc->Z, E = sc->E_el;
    const double *vj = V + (int64_t)j * ldv;
    double *w = V + (int64_t)(j + 1) * ldv;
    const int64_t L = ldv;
    const double gdotv = split ? grad_dot(grad, vj, ncols, sh) : 0.0;
    const double v0 = vj[0];
    double pa = 0.0;
    for (int64_t i = threadIdx.x; i < L; i += kVecThreads) {
        double x = (i < ncols) ? centred_component(i, yH, yS, grad, v0, gdotv, Z, E, split) : 0.0;
        if (mode == IRL_MODE_P && i == 0) x = 0.0;
        w[i] = x;
        pa += vj[i] * x;
    }
    double alpha = block_sum(pa, sh);
    const double bprev = j > 0 ? sc->beta[j - 1] : 0.0;
    for (int64_t i = threadIdx.x; i < L; i += kVecThreads) {
        double x = w[i] - alpha * vj[i];
        if (j > 0) x -= bprev * V[(int64_t)(j - 1) * ldv + i];
        w[i] = x;
    }
    __syncthreads();
    alpha += cgs2(V, ldv, j + 1, w, L, sh, hsh);
    double pb = 0.0;
    for (int64_t i = threadIdx.x; i < L; i += kVecThreads) pb += w[i] * w[i];
    double beta = sqrt(block_sum(pb, sh));
    double normT = fmax(sc->normT, fmax(fabs(alpha), beta));
    if (beta <= 1e3 * 1.1102230246251565e-16 * normT) {
        // invariant subspace: continue with a fresh vector, T decouples
        fresh_vector(V, ldv, j + 1, w, L, ncols, mode, seed ^ (0x5bd1e995ull * (uint64_t)(j + 1 + 64 * sc->breakdowns)), sh, hsh);
        beta = 0.0;
        if (threadIdx.x == 0) sc->breakdowns += 1;
    } else {
        for (int64_t i = threadIdx.x; i < L; i += kVecThreads) w[i] /= beta;
    }
    if (threadIdx.x == 0) {
        sc->alpha[j] = alpha;
        sc->beta[j] = beta;
        sc->normT = normT;
    }
}

__global__ __launch_bounds__(kVecThreads) void k_lanczos_step(
    const double *__restrict__ yH, const double *__restrict__ yS, const double *__restrict__ grad,
    WsScalars *sc, double *V, int64_t ldv, int64_t ncols, int j, int mode, int split, uint64_t seed)
{
    lanczos_step_body(yH, yS, grad, sc, V, ldv, ncols, j, mode, split, seed);
}

hipError_t launch_lanczos_step(const WsLayout &L, void *ws, double *V, int j, int mode, int split,
                               uint64_t seed, hipStream_t st)
{
    k_lanczos_step<<<1, kVecThreads, 0, st>>>(ws_ptr<double>(ws, L.off_yh), ws_ptr<double>(ws, L.off_ys),
                                               ws_ptr<double>(ws, L.off_grad),
                                               ws_ptr<WsScalars>(ws, L.off_scal), V, L.ldv, L.ncols,
                                               j, mode, split, seed);
    return hipGetLastError();
}

// ----------------------------------------------------- tridiagonal QR (one wave)
// d[0..m), e[0..m-1) (e[i] couples i and i+1) in LDS; Z column-major m x m in
// LDS, Z[l + m*i]; lane l updates row l of Z.
__device__ void qr_chase(double *d, double *e, double *Zm, int m, int l, int r, double mu)
{
    const int lane = threadIdx.x;
    double x = d[l] - mu, z = e[l];
    for (int k = l; k < r; ++k) {
        double rr = hypot(x, z);
        double c = rr > 0.0 ? x / rr : 1.0, s = rr > 0.0 ? z / rr : 0.0;
        double dk = d[k], dk1 = d[k + 1], ek = e[k];
        double ek1 = (k + 1 < r) ? e[k + 1] : 0.0;
        __syncthreads();
        if (lane == 0) {
            if (k > l) e[k - 1] = rr;
            d[k] = c * c * dk + 2.0 * c * s * ek + s * s * dk1;
            d[k + 1] = s * s * dk - 2.0 * c * s * ek + c * c * dk1;
            e[k] = c * s * (dk1 - dk) + (c * c - s * s) * ek;
            if (k + 1 < r) e[k + 1] = c * ek1;
        }
        if (lane < m) {
            double zk = Zm[lane + m * k], zk1 = Zm[lane + m * (k + 1)];
            Zm[lane + m * k] = c * zk + s * zk1;
            Zm[lane + m * (k + 1)] = -s * zk + c * zk1;
        }
        __syncthreads();
        if (k + 1 < r) {
            x = e[k];
            z = s * ek1;   // bulge at (k+2, k)
        }
    }
}

__device__ void deflate(double *d, double *e, int m)
{
    __syncthreads();
    if (threadIdx.x == 0)
        for (int i = 0; i + 1 < m; ++i)
            if (fabs(e[i]) <= 1.1102230246251565e-16 * (fabs(d[i]) + fabs(d[i + 1]))) e[i] = 0.0;
    __syncthreads();
}

__device__ void set_identity(double *Zm, int m)
{
    for (int i = threadIdx.x; i < m * m; i += blockDim.x) Zm[i] = (i % m == i / m) ? 1.0 : 0.0;
    __syncthreads();
}

// eigen-decomposition of the symmetric tridiagonal (d, e): d <- eigenvalues,
// Zm <- eigenvectors (columns); Wilkinson-shift implicit QR with deflation.
__device__ void tridiag_eig(double *d, double *e, double *Zm, int m)
{
    set_identity(Zm, m);
    for (int it = 0; it < 60 * m; ++it) {
        deflate(d, e, m);
        int r = m - 1;
        while (r > 0 && e[r - 1] == 0.0) --r;
        if (r == 0) break;
        int l = r - 1;
        while (l > 0 && e[l - 1] != 0.0) --l;
        double a = d[r - 1], c = d[r], b = e[r - 1];
        double del = 0.5 * (a - c);
        double den = del + (del >= 0.0 ? 1.0 : -1.0) * hypot(del, b);
        double mu = den != 0.0 ? c - b * b / den : c;
        qr_chase(d, e, Zm, m, l, r, mu);
    }
}

__device__ void ritz_body(WsScalars *sc, int m, int k)
{
    __shared__ double d[kMaxKrylov], e[kMaxKrylov], Zm[kMaxKrylov * kMaxKrylov];
    __shared__ int rank[kMaxKrylov];
    const int lane = threadIdx.x;
    if (lane < m) {
        d[lane] = sc->alpha[lane];
        e[lane] = lane + 1 < m ? sc->beta[lane] : 0.0;
    }
    __syncthreads();
    tridiag_eig(d, e, Zm, m);
    // ascending order, ties by index
    if (lane < m) {
        int rk = 0;
        for (int t = 0; t < m; ++t) rk += (d[t] < d[lane]) || (d[t] == d[lane] && t < lane);
        rank[lane] = rk;
    }
    __syncthreads();
    if (lane < m) {
        sc->ritz[rank[lane]] = d[lane];
        for (int i = 0; i < m; ++i) sc->U[lane + m * rank[i]] = Zm[lane + m * i];
    }
    __syncthreads();
    if (lane == 0) {
        double lam = sc->ritz[0];
        double nrm = 0.0;
        for (int i = 0; i < m; ++i) nrm = fmax(nrm, fabs(sc->ritz[i]));
        sc->lam = lam;
        sc->gap = m > 1 ? sc->ritz[1] - lam : 0.0;
        sc->resid_est = fabs(sc->beta[m - 1] * sc->U[(m - 1) + m * 0]);
        sc->normT = nrm;
    }
    __syncthreads();
    // implicit restart: m - k exact shifts (largest Ritz values) on the original T
    if (k <= 0 || k >= m) return;
    if (lane < m) {
        d[lane] = sc->alpha[lane];
        e[lane] = lane + 1 < m ? sc->beta[lane] : 0.0;
    }
    __syncthreads();
    set_identity(Zm, m);
    for (int sidx = m - 1; sidx >= k; --sidx) {
        const double mu = sc->ritz[sidx];
        deflate(d, e, m);
        int l = 0;
        while (l < m - 1) {
            if (e[l] == 0.0) { ++l; continue; }
            int r = l;
            while (r < m - 1 && e[r] != 0.0) ++r;
            qr_chase(d, e, Zm, m, l, r, mu);
            l = r + 1;
        }
    }
    __syncthreads();
    if (lane < m) {
        for (int i = 0; i < m; ++i) sc->Q[lane + m * i] = Zm[lane + m * i];
        sc->talpha[lane] = d[lane];
        sc->tbeta[lane] = e[lane];
    }
}

__global__ __launch_bounds__(64) void k_ritz(WsScalars *sc, int m, int k)
{
    ritz_body(sc, m, k);
}

hipError_t launch_ritz(const WsLayout &L, void *ws, int m, int k, hipStream_t st)
{
    k_ritz<<<1, 64, 0, st>>>(ws_ptr<WsScalars>(ws, L.off_scal), m, k);
    return hipGetLastError();
}

// V+ = V Q[:, :k], f = V Q[:, k] * T+[k][k-1] + beta_m Q[m-1][k-1] v_{m+1},
// v_{k+1} = f / ||f|| (reorthogonalised), T <- leading k x k of Q^T T Q.
__device__ void restart_basis_body(WsScalars *sc, const double *Vold,
                                                              double *Vnew, int64_t ldv,
                                                              int64_t ncols, int m, int k, int mode,
                                                              uint64_t seed)
{
    __shared__ double sh[kVecWaves * (kMaxKrylov + 1)];
    __shared__ double hsh[kMaxKrylov + 1];
    __shared__ double Qs[kMaxKrylov * (kMaxKrylov + 1)];
    for (int i = threadIdx.x; i < m * (k + 1); i += kVecThreads) Qs[i] = sc->Q[i];
    __syncthreads();
    const double bk = sc->tbeta[k - 1];
    const double sig = sc->beta[m - 1] * sc->Q[(m - 1) + m * (k - 1)];
    double *f = Vnew + (int64_t)k * ldv;
    for (int64_t c = threadIdx.x; c < ldv; c += kVecThreads) {
        for (int i = 0; i <= k; ++i) {
            double acc = 0.0;
            for (int l = 0; l < m; ++l) acc += Vold[(int64_t)l * ldv + c] * Qs[l + m * i];
            if (i < k)
                Vnew[(int64_t)i * ldv + c] = acc;
            else
                f[c] = acc * bk + sig * Vold[(int64_t)m * ldv + c];
        }
    }
    __syncthreads();
    cgs2(Vnew, ldv, k, f, ldv, sh, hsh);
    double p = 0.0;
    for (int64_t c = threadIdx.x; c < ldv; c += kVecThreads) p += f[c] * f[c];
    double nrm = sqrt(block_sum(p, sh));
    double normT = 0.0;
    for (int i = 0; i < k; ++i) normT = fmax(normT, fabs(sc->talpha[i]));
    for (int i = 0; i + 1 < k; ++i) normT = fmax(normT, fabs(sc->tbeta[i]));
    normT = fmax(normT, nrm);
    if (nrm <= 1e3 * 1.1102230246251565e-16 * normT) {
        fresh_vector(Vnew, ldv, k, f, ldv, ncols, mode, seed ^ 0x27d4eb2f165667c5ull, sh, hsh);
        nrm = 0.0;
    } else {
        for (int64_t c = threadIdx.x; c < ldv; c += kVecThreads) f[c] /= nrm;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 0; i < k; ++i) sc->alpha[i] = sc->talpha[i];
        for (int i = 0; i + 1 < k; ++i) sc->beta[i] = sc->tbeta[i];
        sc->beta[k - 1] = nrm;
        sc->normT = normT;
    }
}

__global__ __launch_bounds__(kVecThreads) void k_restart_basis(WsScalars *sc, const double *Vold,
                                                              double *Vnew, int64_t ldv,
                                                              int64_t ncols, int m, int k, int mode,
                                                              uint64_t seed)
{
    restart_basis_body(sc, Vold, Vnew, ldv, ncols, m, k, mode, seed);
}

hipError_t launch_restart_basis(const WsLayout &L, void *ws, const double *Vold, double *Vnew,
                                int m, int k, int mode, uint64_t seed, hipStream_t st)
{
    k_restart_basis<<<1, kVecThreads, 0, st>>>(ws_ptr<WsScalars>(ws, L.off_scal), Vold, Vnew, L.ldv,
                                               L.ncols, m, k, mode, seed);
    return hipGetLastError();
}

// y = V U[:, 0] normalised; c0 = y[0]
__device__ void ritz_vector_body(WsScalars *sc, const double *V,
                                                            int64_t ldv, int m, double *y)
{
    __shared__ double sh[kVecWaves * (kMaxKrylov + 1)];
    double p = 0.0;
    for (int64_t c = threadIdx.x; c < ldv; c += kVecThreads) {
        double acc = 0.0;
        for (int l = 0; l < m; ++l) acc += V[(int64_t)l * ldv + c] * sc->U[l];
        y[c] = acc;
        p += acc * acc;
    }
    double nrm = sqrt(block_sum(p, sh));
    for (int64_t c = threadIdx.x; c < ldv; c += kVecThreads) y[c] /= nrm;
    __syncthreads();
    if (threadIdx.x == 0) sc->c0 = y[0];
}

__global__ __launch_bounds__(kVecThreads) void k_ritz_vector(WsScalars *sc, const double *V,
                                                            int64_t ldv, int m, double *y)
{
    ritz_vector_body(sc, V, ldv, m, y);
}

hipError_t launch_ritz_vector(const WsLayout &L, void *ws, const double *V, int m, double *y,
                              hipStream_t st)
{
    k_ritz_vector<<<1, kVecThreads, 0, st>>>(ws_ptr<WsScalars>(ws, L.off_scal), V, L.ldv, m, y);
    return hipGetLastError();
}

// r = H~'y - lam y from (yH, yS); resid2 = ||r||^2
__device__ void residual_body(WsScalars *sc, const double *yH,
                                                         const double *yS, const double *grad,
                                                         const double *y, double *r, int64_t ldv,
                                                         int64_t ncols, int mode, int split)
{
    __shared__ double sh[kVecWaves * (kMaxKrylov + 1)];
    const double Z = sc->Z, E = sc->E_el, lam = sc->lam;
    const double gdotv = split ? grad_dot(grad, y, ncols, sh) : 0.0;
    const double v0 = y[0];
    double p = 0.0;
    for (int64_t c = threadIdx.x; c < ldv; c += kVecThreads) {
        double x = c < ncols ? centred_component(c, yH, yS, grad, v0, gdotv, Z, E, split) - lam * y[c]
                             : 0.0;
        if (mode == IRL_MODE_P && c == 0) x = 0.0;
        r[c] = x;
        p += x * x;
    }
    double s = block_sum(p, sh);
    if (threadIdx.x == 0) sc->resid2 = s;
}

__global__ __launch_bounds__(kVecThreads) void k_residual(WsScalars *sc, const double *yH,
                                                         const double *yS, const double *grad,
                                                         const double *y, double *r, int64_t ldv,
                                                         int64_t ncols, int mode, int split)
{
    residual_body(sc, yH, yS, grad, y, r, ldv, ncols, mode, split);
}

hipError_t launch_residual(const WsLayout &L, void *ws, const double *y, double *r, int mode,
                           int split, hipStream_t st)
{
    k_residual<<<1, kVecThreads, 0, st>>>(ws_ptr<WsScalars>(ws, L.off_scal),
                                          ws_ptr<double>(ws, L.off_yh), ws_ptr<double>(ws, L.off_ys),
                                          ws_ptr<double>(ws, L.off_grad), y, r, L.ldv, L.ncols, mode,
                                          split);
    return hipGetLastError();
}

// dtheta = y[1:] / y[0]; theta += dtheta
__global__ void k_update(const double *y, double *dtheta, double *theta, int64_t P)
{
    const double c0 = y[0];
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < P;
         i += (int64_t)gridDim.x * blockDim.x) {
        double d = y[i + 1] / c0;
        if (dtheta) dtheta[i] = d;
        if (theta) theta[i] += d;
    }
}

hipError_t launch_update(const WsLayout &, void *, const double *y, double *dtheta, double *theta,
                         int64_t P, int, hipStream_t st)
{
    unsigned blocks = (unsigned)((P + 255) / 256);
    if (blocks > 1024) blocks = 1024;
    k_update<<<blocks, 256, 0, st>>>(y, dtheta, theta, P);
    return hipGetLastError();
}

__global__ void k_copy(double *dst, const double *src, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

hipError_t launch_copy(double *dst, const double *src, int64_t n, hipStream_t st)
{
    unsigned blocks = (unsigned)((n + 255) / 256);
    if (blocks > 2048) blocks = 2048;
    if (blocks == 0) return hipSuccess;
    k_copy<<<blocks, 256, 0, st>>>(dst, src, n);
    return hipGetLastError();
}

}  // namespace irl

namespace irl {

__global__ void k_reset_solve(WsScalars *sc)
{
    if (threadIdx.x == 0) {
        sc->normT = 0.0;
        sc->breakdowns = 0;
        sc->resid2 = 0.0;
    }
}

hipError_t launch_reset_solve(const WsLayout &L, void *ws, hipStream_t st)
{
    k_reset_solve<<<1, 64, 0, st>>>(ws_ptr<WsScalars>(ws, L.off_scal));
    return hipGetLastError();
}

}  // namespace irl

// ---------------------------------------------------------------------------
// Grouped launches for a batch of independent systems advancing in lockstep:
// block b works on member items[b].m with exactly the per-member arithmetic of
// the solo kernels above.
// ---------------------------------------------------------------------------
namespace irl {

__global__ void k_reset_grouped(const Member *__restrict__ M, const WorkItem *__restrict__ items)
{
    if (threadIdx.x == 0) {
        WsScalars *sc = M[items[blockIdx.x].m].sc;
        sc->normT = 0.0;
        sc->breakdowns = 0;
        sc->resid2 = 0.0;
    }
}

__global__ __launch_bounds__(kVecThreads) void k_start_vector_grouped(
    const Member *__restrict__ M, const WorkItem *__restrict__ items, int mode, uint64_t seed,
    int from_y)
{
    __shared__ double sh[kVecWaves * (kMaxKrylov + 1)];
    __shared__ double hsh[kMaxKrylov + 1];
    const Member &mb = M[items[blockIdx.x].m];
    if (from_y) {
        for (int64_t i = threadIdx.x; i < mb.ld; i += kVecThreads) mb.kry[0][i] = mb.y[i];
        return;
    }
    fresh_vector(nullptr, mb.ld, 0, mb.kry[0], mb.ld, mb.ncols, mode, seed, sh, hsh);
}

__global__ __launch_bounds__(kVecThreads) void k_lanczos_step_grouped(
    const Member *__restrict__ M, const WorkItem *__restrict__ items, int j, int cur, int mode,
    int split, uint64_t seed)
{
    const Member &mb = M[items[blockIdx.x].m];
    lanczos_step_body(mb.yH, mb.yS, mb.grad, mb.sc, mb.kry[cur], mb.ld, mb.ncols, j, mode, split,
                      seed);
}

__global__ __launch_bounds__(64) void k_ritz_grouped(const Member *__restrict__ M,
                                                     const WorkItem *__restrict__ items, int m,
                                                     int k)
{
    ritz_body(M[items[blockIdx.x].m].sc, m, k);
}

__global__ __launch_bounds__(kVecThreads) void k_restart_basis_grouped(
    const Member *__restrict__ M, const WorkItem *__restrict__ items, int cur, int m, int k,
    int mode, uint64_t seed)
{
    const Member &mb = M[items[blockIdx.x].m];
    restart_basis_body(mb.sc, mb.kry[cur], mb.kry[1 - cur], mb.ld, mb.ncols, m, k, mode, seed);
}

__global__ __launch_bounds__(kVecThreads) void k_ritz_vector_grouped(
    const Member *__restrict__ M, const WorkItem *__restrict__ items, int cur, int m)
{
    const Member &mb = M[items[blockIdx.x].m];
    ritz_vector_body(mb.sc, mb.kry[cur], mb.ld, m, mb.y);
}

__global__ __launch_bounds__(kVecThreads) void k_residual_grouped(
    const Member *__restrict__ M, const WorkItem *__restrict__ items, int mode, int split)
{
    const Member &mb = M[items[blockIdx.x].m];
    residual_body(mb.sc, mb.yH, mb.yS, mb.grad, mb.y, mb.r, mb.ld, mb.ncols, mode, split);
}

__global__ void k_update_grouped(const Member *__restrict__ M, const WorkItem *__restrict__ items)
{
    const Member &mb = M[items[blockIdx.x].m];
    const double c0 = mb.y[0];
    for (int64_t i = threadIdx.x; i < mb.ncols - 1; i += blockDim.x) {
        const double d = mb.y[i + 1] / c0;
        if (mb.dtheta) mb.dtheta[i] = d;
        if (mb.theta) mb.theta[i] += d;
    }
}

__global__ void k_gather_scalars(const Member *__restrict__ M, const WorkItem *__restrict__ items,
                                 MemberScalars *out)
{
    if (threadIdx.x != 0) return;
    const int m = items[blockIdx.x].m;
    const WsScalars *sc = M[m].sc;
    MemberScalars o;
    o.Z = sc->Z;
    o.E_el = sc->E_el;
    o.lam = sc->lam;
    o.resid_est = sc->resid_est;
    o.gap = sc->gap;
    o.normT = sc->normT;
    o.c0 = sc->c0;
    o.resid2 = sc->resid2;
    out[m] = o;
}

hipError_t launch_lanczos_grouped(int op, const Member *M, const WorkItem *items, int nitems,
                                  int i0, int i1, int i2, int i3, uint64_t seed,
                                  MemberScalars *out, hipStream_t st)
{
    if (nitems <= 0) return hipSuccess;
    switch (op) {
    case kGrpReset: k_reset_grouped<<<nitems, 64, 0, st>>>(M, items); break;
    case kGrpStart: k_start_vector_grouped<<<nitems, kVecThreads, 0, st>>>(M, items, i0, seed, i1); break;
    case kGrpLanczos: k_lanczos_step_grouped<<<nitems, kVecThreads, 0, st>>>(M, items, i0, i1, i2, i3, seed); break;
    case kGrpRitz: k_ritz_grouped<<<nitems, 64, 0, st>>>(M, items, i0, i1); break;
    case kGrpRestart: k_restart_basis_grouped<<<nitems, kVecThreads, 0, st>>>(M, items, i0, i1, i2, i3, seed); break;
    case kGrpRitzVector: k_ritz_vector_grouped<<<nitems, kVecThreads, 0, st>>>(M, items, i0, i1); break;
    case kGrpResidual: k_residual_grouped<<<nitems, kVecThreads, 0, st>>>(M, items, i0, i1); break;
    case kGrpUpdate: k_update_grouped<<<nitems, 256, 0, st>>>(M, items); break;
    case kGrpGather: k_gather_scalars<<<nitems, 64, 0, st>>>(M, items, out); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace irl
