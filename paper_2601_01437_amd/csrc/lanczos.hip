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
// img (column j of the image basis): a copy of H~' v_j, so that the image of any
// combination of basis vectors (a Ritz vector) is the same combination of images.
// sig (mode C only, else null): D~^T psi.  The connected basis adds
// -(g_i sigma.v + sigma_i g.v) / 2 to components i >= 1, sigma = sig / Z.
__device__ void lanczos_step_body(
    const double *__restrict__ yH, const double *__restrict__ yS, const double *__restrict__ grad,
    const double *__restrict__ sig, WsScalars *sc, double *V, double *img, int64_t ldv, int64_t ncols,
    int j, int mode, int split, uint64_t seed)
{
    __shared__ double sh[kVecWaves * (kMaxKrylov + 1)];
    __shared__ double hsh[kMaxKrylov + 1];
    const double Z = sc->Z, E = sc->E_el;
    // this cycle's seed: the solve's seed advanced by the restarts done so far
    const uint64_t sd = seed + 0x100000001b3ull * (uint64_t)(sc->restarts + 1);
    const double *vj = V + (int64_t)j * ldv;
    double *w = V + (int64_t)(j + 1) * ldv;
    const int64_t L = ldv;
    const double gdotv = (split || sig) ? grad_dot(grad, vj, ncols, sh) : 0.0;
    const double sdotv = sig ? grad_dot(sig, vj, ncols, sh) / Z : 0.0;
    const double v0 = vj[0];
    double pa = 0.0;
    for (int64_t i = threadIdx.x; i < L; i += kVecThreads) {
        double x = (i < ncols) ? centred_component(i, yH, yS, grad, v0, gdotv, Z, E, split) : 0.0;
        if (sig && i >= 1 && i < ncols) x -= 0.5 * (grad[i] * sdotv + (sig[i] / Z) * gdotv);
        if (mode == IRL_MODE_P && i == 0) x = 0.0;
        w[i] = x;
        img[(int64_t)j * ldv + i] = x;
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
        fresh_vector(V, ldv, j + 1, w, L, ncols, mode, sd ^ (0x5bd1e995ull * (uint64_t)(j + 1 + 64 * sc->breakdowns)), sh, hsh);
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
    const double *__restrict__ sig, WsScalars *sc, double *V, double *img, int64_t ldv, int64_t ncols,
    int j, int mode, int split, uint64_t seed)
{
    lanczos_step_body(yH, yS, grad, sig, sc, V, img, ldv, ncols, j, mode, split, seed);
}

hipError_t launch_lanczos_step(const WsLayout &L, void *ws, double *V, double *img, int j, int mode,
                               int split, uint64_t seed, hipStream_t st)
{
    const double *sig = mode == IRL_MODE_C ? ws_ptr<double>(ws, L.off_sig) : nullptr;
    k_lanczos_step<<<1, kVecThreads, 0, st>>>(ws_ptr<double>(ws, L.off_yh), ws_ptr<double>(ws, L.off_ys),
                                               ws_ptr<double>(ws, L.off_grad), sig,
                                               ws_ptr<WsScalars>(ws, L.off_scal), V, img, L.ldv, L.ncols,
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
__device__ void restart_basis_body(WsScalars *sc, const double *Vold, double *Vnew,
                                   const double *Iold, double *Inew, int64_t ldv, int64_t ncols,
                                   int m, int k, int mode, uint64_t seed)
{
    __shared__ double sh[kVecWaves * (kMaxKrylov + 1)];
    __shared__ double hsh[kMaxKrylov + 1];
    __shared__ double Qs[kMaxKrylov * (kMaxKrylov + 1)];
    const uint64_t sd = seed ^ (0x9e3779b97f4a7c15ull * (uint64_t)(sc->restarts + 7));
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
        // images of the kept vectors: the same combinations of the old images
        for (int i = 0; i < k; ++i) {
            double acc = 0.0;
            for (int l = 0; l < m; ++l) acc += Iold[(int64_t)l * ldv + c] * Qs[l + m * i];
            Inew[(int64_t)i * ldv + c] = acc;
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
        fresh_vector(Vnew, ldv, k, f, ldv, ncols, mode, sd ^ 0x27d4eb2f165667c5ull, sh, hsh);
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
        sc->restarts += 1;
    }
}

__global__ __launch_bounds__(kVecThreads) void k_restart_basis(WsScalars *sc, const double *Vold,
                                                              double *Vnew, const double *Iold,
                                                              double *Inew, int64_t ldv, int64_t ncols,
                                                              int m, int k, int mode, uint64_t seed)
{
    restart_basis_body(sc, Vold, Vnew, Iold, Inew, ldv, ncols, m, k, mode, seed);
}

hipError_t launch_restart_basis(const WsLayout &L, void *ws, const double *Vold, double *Vnew,
                                const double *Iold, double *Inew, int m, int k, int mode, uint64_t seed,
                                hipStream_t st)
{
    k_restart_basis<<<1, kVecThreads, 0, st>>>(ws_ptr<WsScalars>(ws, L.off_scal), Vold, Vnew, Iold, Inew,
                                               L.ldv, L.ncols, m, k, mode, seed);
    return hipGetLastError();
}

// y = V U[:, 0] normalised, c0 = y[0]; hy = img U[:, 0] with the same scale:
// the operator image of y, formed from the images of the basis vectors
__device__ void ritz_vector_body(WsScalars *sc, const double *V, const double *img, int64_t ldv,
                                 int m, double *y, double *hy)
{
    __shared__ double sh[kVecWaves * (kMaxKrylov + 1)];
    double p = 0.0;
    for (int64_t c = threadIdx.x; c < ldv; c += kVecThreads) {
        double acc = 0.0, acch = 0.0;
        for (int l = 0; l < m; ++l) {
            acc += V[(int64_t)l * ldv + c] * sc->U[l];
            acch += img[(int64_t)l * ldv + c] * sc->U[l];
        }
        y[c] = acc;
        hy[c] = acch;
        p += acc * acc;
    }
    double nrm = sqrt(block_sum(p, sh));
    for (int64_t c = threadIdx.x; c < ldv; c += kVecThreads) {
        y[c] /= nrm;
        hy[c] /= nrm;
    }
    __syncthreads();
    if (threadIdx.x == 0) sc->c0 = y[0];
}

__global__ __launch_bounds__(kVecThreads) void k_ritz_vector(WsScalars *sc, const double *V,
                                                            const double *img, int64_t ldv, int m,
                                                            double *y, double *hy)
{
    ritz_vector_body(sc, V, img, ldv, m, y, hy);
}

hipError_t launch_ritz_vector(const WsLayout &L, void *ws, const double *V, const double *img, int m,
                              double *y, double *hy, hipStream_t st)
{
    k_ritz_vector<<<1, kVecThreads, 0, st>>>(ws_ptr<WsScalars>(ws, L.off_scal), V, img, L.ldv, m, y, hy);
    return hipGetLastError();
}

// r = hy - lam y with hy = H~' y; resid2 = ||r||^2
__device__ void residual_image_body(WsScalars *sc, const double *y, const double *hy, double *r,
                                    int64_t ldv, int mode)
{
    __shared__ double sh[kVecWaves * (kMaxKrylov + 1)];
    const double lam = sc->lam;
    double p = 0.0;
    for (int64_t c = threadIdx.x; c < ldv; c += kVecThreads) {
        double x = hy[c] - lam * y[c];
        if (mode == IRL_MODE_P && c == 0) x = 0.0;
        r[c] = x;
        p += x * x;
    }
    const double s = block_sum(p, sh);
    if (threadIdx.x == 0) sc->resid2 = s;
}

__global__ __launch_bounds__(kVecThreads) void k_residual_image(WsScalars *sc, const double *y,
                                                               const double *hy, double *r, int64_t ldv,
                                                               int mode)
{
    residual_image_body(sc, y, hy, r, ldv, mode);
}

hipError_t launch_residual_image(const WsLayout &L, void *ws, const double *y, const double *hy, double *r,
                                 int mode, hipStream_t st)
{
    k_residual_image<<<1, kVecThreads, 0, st>>>(ws_ptr<WsScalars>(ws, L.off_scal), y, hy, r, L.ldv, mode);
    return hipGetLastError();
}

// dtheta = y[1:] / *c0p; theta += dtheta.  c0p is y[0] (mode A) or the connected
// basis' coefficient of psi (mode C).
__global__ void k_update(const double *y, const double *c0p, double *dtheta, double *theta, int64_t P)
{
    const double c0 = *c0p;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < P;
         i += (int64_t)gridDim.x * blockDim.x) {
        double d = y[i + 1] / c0;
        if (dtheta) dtheta[i] = d;
        if (theta) theta[i] += d;
    }
}

// Adam (bias-corrected first and second moments), elementwise over the P parameters
__global__ void k_adam(double *__restrict__ theta, const double *__restrict__ g, double *__restrict__ m,
                       double *__restrict__ v, int64_t P, double lr, double b1, double b2, double eps,
                       double c1, double c2)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P) return;
    const double gi = g[i];
    const double mi = b1 * m[i] + (1.0 - b1) * gi;
    const double vi = b2 * v[i] + (1.0 - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    theta[i] -= lr * (mi / c1) / (sqrt(vi / c2) + eps);
}

hipError_t launch_adam(double *theta, const double *g, double *m, double *v, int64_t P, double lr, double b1,
                       double b2, double eps, int64_t t, hipStream_t st)
{
    const double c1 = 1.0 - pow(b1, (double)t), c2 = 1.0 - pow(b2, (double)t);
    k_adam<<<(unsigned)((P + 255) / 256), 256, 0, st>>>(theta, g, m, v, P, lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}

hipError_t launch_update(const WsLayout &L, void *ws, const double *y, double *dtheta, double *theta,
                         int64_t P, int mode, hipStream_t st)
{
    unsigned blocks = (unsigned)((P + 255) / 256);
    if (blocks > 1024) blocks = 1024;
    const double *c0p = mode == IRL_MODE_C ? &ws_ptr<WsScalars>(ws, L.off_scal)->c0 : y;
    k_update<<<blocks, 256, 0, st>>>(y, c0p, dtheta, theta, P);
    return hipGetLastError();
}

// connected basis: the coefficient of psi in the linearised wavefunction,
// c0 = y[0] - sum_{i >= 1} sig[i] y[i] / Z, into sc->c0 (one block, fixed order)
__global__ __launch_bounds__(kVecThreads) void k_connected_c0(WsScalars *sc, const double *__restrict__ y,
                                                             const double *__restrict__ sig, int64_t ncols)
{
    __shared__ double sh[kVecWaves];
    const double s = grad_dot(sig, y, ncols, sh);
    if (threadIdx.x == 0) sc->c0 = y[0] - s / sc->Z;
}

hipError_t launch_connected_c0(const WsLayout &L, void *ws, const double *y, hipStream_t st)
{
    k_connected_c0<<<1, kVecThreads, 0, st>>>(ws_ptr<WsScalars>(ws, L.off_scal), y,
                                              ws_ptr<double>(ws, L.off_sig), L.ncols);
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
        sc->restarts = 0;
        sc->resid2 = 0.0;
    }
}

hipError_t launch_reset_solve(const WsLayout &L, void *ws, hipStream_t st)
{
    k_reset_solve<<<1, 64, 0, st>>>(ws_ptr<WsScalars>(ws, L.off_scal));
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Thick-restart block Lanczos (the block variant the paper names as its future
// direction, Discussion): nb vectors per operator pass.  Basis Q (orthonormal
// columns), projected matrix T = Q^T H~' Q kept in full (row-major, leading
// dimension kBasisCols) so that T stays exact after thick restarts:
//   step:     Z = H~' Q_J for the newest block J; T[:, J] = Q^T Z (two passes of
//             classical Gram-Schmidt against all columns); Z = Q_next R by
//             modified Gram-Schmidt (two passes) inside the block; T[next, J] = R;
//   Ritz:     T_s = Y Theta Y^T (Householder tridiagonalisation + the implicit
//             QR of the single-vector path); residual of pair i = ||C y_i|| with
//             C = T[next, 0:s], the coupling of the pending block;
//   restart:  Q <- [Q Y_k, Q_next], T <- [[Theta_k, E^T], [E, .]], E = C Y_k
//             (equivalent to exact-shift implicit restarts, Algorithm 1, for nb = 1).
constexpr int kTld = kBasisCols;
constexpr int kBSh = kBasisCols + 1;

// h[d] = V[d] . w for d < nd (fixed order), into shared hsh[nd]; nd <= kBasisCols
__device__ void bdots(const double *V, int64_t ldv, int nd, const double *w, int64_t L, double *sh,
                      double *hsh)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    __syncthreads();
    for (int d = 0; d < nd; ++d) {
        double p = 0.0;
        for (int64_t i = threadIdx.x; i < L; i += kVecThreads) p += V[d * ldv + i] * w[i];
        for (int off = 32; off > 0; off >>= 1) p += __shfl_xor(p, off, kWave);
        if (lane == 0) sh[wv * kBSh + d] = p;
    }
    __syncthreads();
    if (threadIdx.x < nd) {
        double s = 0.0;
        for (int i = 0; i < kVecWaves; ++i) s += sh[i * kBSh + threadIdx.x];
        hsh[threadIdx.x] = s;
    }
    __syncthreads();
}

// two passes of classical Gram-Schmidt of w against V[0..nd); coef[d] += both passes
__device__ void bcgs2(const double *V, int64_t ldv, int nd, double *w, int64_t L, double *sh, double *hsh,
                      double *coef)
{
    for (int pass = 0; pass < 2; ++pass) {
        bdots(V, ldv, nd, w, L, sh, hsh);
        if (coef && threadIdx.x < nd) coef[threadIdx.x] += hsh[threadIdx.x];
        block_sub(V, ldv, nd, hsh, w, L);
    }
}

__device__ double bnorm(const double *w, int64_t L, double *sh)
{
    double p = 0.0;
    for (int64_t i = threadIdx.x; i < L; i += kVecThreads) p += w[i] * w[i];
    return sqrt(block_sum(p, sh));
}

// random unit vector orthogonal to V[0..nd) into w (component 0 zero in mode P)
__device__ void bfresh(const double *V, int64_t ldv, int nd, double *w, int64_t L, int64_t ncols, int mode,
                       uint64_t seed, double *sh, double *hsh)
{
    for (int64_t i = threadIdx.x; i < L; i += kVecThreads)
        w[i] = (i < ncols && !(mode == IRL_MODE_P && i == 0)) ? uniform_pm1(seed, (uint64_t)i) : 0.0;
    __syncthreads();
    bcgs2(V, ldv, nd, w, L, sh, hsh, nullptr);
    const double nrm = bnorm(w, L, sh);
    for (int64_t i = threadIdx.x; i < L; i += kVecThreads) w[i] = nrm > 0.0 ? w[i] / nrm : 0.0;
    __syncthreads();
}

// start block: nb orthonormal random vectors in columns [0, nb); T cleared
__global__ __launch_bounds__(kVecThreads) void k_block_start(WsScalars *sc, double *V, int64_t ldv,
                                                            int64_t ncols, int nb, int mode, uint64_t seed)
{
    __shared__ double sh[kVecWaves * kBSh];
    __shared__ double hsh[kBSh];
    for (int i = threadIdx.x; i < kTld * kTld; i += kVecThreads) sc->T[i] = 0.0;
    if (threadIdx.x == 0) {
        sc->normT = 0.0;
        sc->breakdowns = 0;
        sc->resid2 = 0.0;
    }
    __syncthreads();
    for (int q = 0; q < nb; ++q)
        bfresh(V, ldv, q, V + (int64_t)q * ldv, ldv, ncols, mode, seed + 0x9E3779B97F4A7C15ull * (uint64_t)q,
               sh, hsh);
}

hipError_t launch_block_start(const WsLayout &L, void *ws, double *V, int nb, int mode, uint64_t seed,
                              hipStream_t st)
{
    if (nb < 1 || nb > kMaxBlock) return hipErrorInvalidValue;
    k_block_start<<<1, kVecThreads, 0, st>>>(ws_ptr<WsScalars>(ws, L.off_scal), V, L.ldv, L.ncols, nb, mode,
                                             seed);
    return hipGetLastError();
}

// One block step on the block in columns [s0, s0 + nb): (yH, yS) hold the raw
// operator pairs of those columns (stride ldy); the next block is written to
// columns [s0 + nb, s0 + 2 nb).
__global__ __launch_bounds__(kVecThreads) void k_block_step(
    const double *__restrict__ yH, const double *__restrict__ yS, int64_t ldy,
    const double *__restrict__ grad, WsScalars *sc, double *V, double *img, int64_t ldv, int64_t ncols,
    int s0, int nb, int mode, int split, uint64_t seed)
{
    __shared__ double sh[kVecWaves * kBSh];
    __shared__ double hsh[kBSh];
    __shared__ double coef[kBSh];
    __shared__ double R[kMaxBlock * kMaxBlock];
    const int64_t L = ldv;
    const double Z = sc->Z, E = sc->E_el;
    // 1. centred images H~' q into the next block's columns
    for (int q = 0; q < nb; ++q) {
        const double *vq = V + (int64_t)(s0 + q) * ldv;
        double *z = V + (int64_t)(s0 + nb + q) * ldv;
        const double gdotv = split ? grad_dot(grad, vq, ncols, sh) : 0.0;
        const double v0 = vq[0];
        for (int64_t i = threadIdx.x; i < L; i += kVecThreads) {
            double x = (i < ncols) ? centred_component(i, yH + q * ldy, yS + q * ldy, grad, v0, gdotv, Z, E,
                                                       split)
                                   : 0.0;
            if (mode == IRL_MODE_P && i == 0) x = 0.0;
            z[i] = x;
            img[(int64_t)(s0 + q) * ldv + i] = x;
        }
        __syncthreads();
    }
    // 2. projection on all columns [0, s0 + nb): T[:, s0 + q]
    const int nd = s0 + nb;
    for (int q = 0; q < nb; ++q) {
        double *z = V + (int64_t)(s0 + nb + q) * ldv;
        if (threadIdx.x < nd) coef[threadIdx.x] = 0.0;
        __syncthreads();
        bcgs2(V, ldv, nd, z, L, sh, hsh, coef);
        __syncthreads();
        if (threadIdx.x < nd) sc->T[threadIdx.x * kTld + (s0 + q)] = coef[threadIdx.x];
        __syncthreads();
    }
    double normT = sc->normT;
    for (int d = 0; d < nd; ++d)
        for (int q = 0; q < nb; ++q) normT = fmax(normT, fabs(sc->T[d * kTld + s0 + q]));
    // 3. orthonormalise the new block in place (two passes of modified Gram-Schmidt)
    for (int q = 0; q < nb; ++q) {
        double *z = V + (int64_t)(s0 + nb + q) * ldv;
        if (threadIdx.x < kMaxBlock) coef[threadIdx.x] = 0.0;
        __syncthreads();
        if (q > 0) bcgs2(V + (int64_t)(s0 + nb) * ldv, ldv, q, z, L, sh, hsh, coef);
        const double nrm = bnorm(z, L, sh);
        double rqq;
        if (nrm <= 1e3 * 1.1102230246251565e-16 * normT) {
            // invariant subspace: continue with a fresh direction, T decouples
            bfresh(V, ldv, s0 + nb + q, z, L, ncols, mode,
                   seed ^ (0x5bd1e995ull * (uint64_t)(s0 + nb + q + 1 + 97 * sc->breakdowns)), sh, hsh);
            rqq = 0.0;
            if (threadIdx.x == 0) sc->breakdowns += 1;
        } else {
            for (int64_t i = threadIdx.x; i < L; i += kVecThreads) z[i] /= nrm;
            rqq = nrm;
        }
        if (threadIdx.x == 0) {
            for (int c = 0; c < kMaxBlock; ++c) R[c * kMaxBlock + q] = c < q ? coef[c] : (c == q ? rqq : 0.0);
        }
        __syncthreads();
    }
    // 4. coupling of the next block (R, upper triangular) and symmetry of T
    for (int idx = threadIdx.x; idx < nb * nb; idx += kVecThreads) {
        const int r = idx / nb, c = idx - r * nb;
        const double val = r <= c ? R[r * kMaxBlock + c] : 0.0;
        sc->T[(s0 + nb + r) * kTld + s0 + c] = val;
        sc->T[(s0 + c) * kTld + s0 + nb + r] = val;
    }
    for (int idx = threadIdx.x; idx < s0 * nb; idx += kVecThreads) {
        const int d = idx / nb, q = idx - d * nb;
        sc->T[(s0 + q) * kTld + d] = sc->T[d * kTld + s0 + q];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 0; i < nb; ++i)
            for (int j = i + 1; j < nb; ++j) {
                const double a = 0.5 * (sc->T[(s0 + i) * kTld + s0 + j] + sc->T[(s0 + j) * kTld + s0 + i]);
                sc->T[(s0 + i) * kTld + s0 + j] = a;
                sc->T[(s0 + j) * kTld + s0 + i] = a;
            }
        for (int r = 0; r < nb; ++r)
            for (int c = 0; c < nb; ++c) normT = fmax(normT, fabs(R[r * kMaxBlock + c]));
        sc->normT = normT;
    }
}

hipError_t launch_block_step(const WsLayout &L, void *ws, double *V, double *img, int s0, int nb, int mode,
                             int split, uint64_t seed, hipStream_t st)
{
    if (nb < 1 || nb > kMaxBlock || s0 < 0 || s0 + 2 * nb > kBasisCols || s0 + nb > kMaxKrylov)
        return hipErrorInvalidValue;
    k_block_step<<<1, kVecThreads, 0, st>>>(ws_ptr<double>(ws, L.off_yh), ws_ptr<double>(ws, L.off_ys), L.ldv,
                                            ws_ptr<double>(ws, L.off_grad), ws_ptr<WsScalars>(ws, L.off_scal),
                                            V, img, L.ldv, L.ncols, s0, nb, mode, split, seed);
    return hipGetLastError();
}

// Ritz pairs of T[0:s, 0:s] (one wavefront): Householder reduction to
// tridiagonal form with the reflections accumulated, the tridiagonal QR of the
// single-vector path, back-transformation; ascending order into ritz / U
// (column-major, leading dimension s); residual estimate of the lowest pair.
__global__ __launch_bounds__(64) void k_block_ritz(WsScalars *sc, int s, int nb)
{
    __shared__ double A[kMaxKrylov * kMaxKrylov];   // T (row-major, ld s), then the QR eigenvectors
    __shared__ double Qh[kMaxKrylov * kMaxKrylov];  // accumulated reflections (row-major, ld s)
    __shared__ double v[kMaxKrylov], p[kMaxKrylov], d[kMaxKrylov], e[kMaxKrylov];
    __shared__ int rank[kMaxKrylov];
    __shared__ double red[kMaxBlock];
    const int lane = threadIdx.x;
    for (int idx = lane; idx < s * s; idx += 64) {
        const int i = idx / s, j = idx - i * s;
        A[idx] = sc->T[i * kTld + j];
        Qh[idx] = (i == j) ? 1.0 : 0.0;
    }
    __syncthreads();
    for (int k = 0; k + 2 < s; ++k) {
        if (lane == 0) {
            double nrm2 = 0.0;
            for (int i = k + 1; i < s; ++i) nrm2 += A[i * s + k] * A[i * s + k];
            const double nrm = sqrt(nrm2);
            const double x0 = A[(k + 1) * s + k];
            const double alpha = x0 >= 0.0 ? -nrm : nrm;
            double vn2 = 0.0;
            for (int i = 0; i < s; ++i) {
                double vi = i > k ? A[i * s + k] : 0.0;
                if (i == k + 1) vi -= alpha;
                v[i] = vi;
                vn2 += vi * vi;
            }
            const double vn = sqrt(vn2);
            for (int i = 0; i < s; ++i) v[i] = vn > 0.0 ? v[i] / vn : 0.0;
        }
        __syncthreads();
        if (lane < s) {
            double acc = 0.0;
            for (int j = k + 1; j < s; ++j) acc += A[lane * s + j] * v[j];
            p[lane] = acc;
        }
        __syncthreads();
        double K = 0.0;
        for (int j = k + 1; j < s; ++j) K += v[j] * p[j];
        // w = 2p - 2K v (into p); A <- A - v w^T - w v^T
        __syncthreads();
        if (lane < s) p[lane] = 2.0 * p[lane] - 2.0 * K * v[lane];
        __syncthreads();
        if (lane < s) {
            for (int j = 0; j < s; ++j) A[lane * s + j] -= v[lane] * p[j] + p[lane] * v[j];
            double t = 0.0;
            for (int l = k + 1; l < s; ++l) t += Qh[lane * s + l] * v[l];
            for (int j = k + 1; j < s; ++j) Qh[lane * s + j] -= 2.0 * t * v[j];
        }
        __syncthreads();
    }
    if (lane < s) {
        d[lane] = A[lane * s + lane];
        e[lane] = lane + 1 < s ? 0.5 * (A[lane * s + lane + 1] + A[(lane + 1) * s + lane]) : 0.0;
    }
    __syncthreads();
    tridiag_eig(d, e, A, s);   // A <- eigenvectors of the tridiagonal (column-major, ld s)
    if (lane < s) {
        int rk = 0;
        for (int t = 0; t < s; ++t) rk += (d[t] < d[lane]) || (d[t] == d[lane] && t < lane);
        rank[lane] = rk;
    }
    __syncthreads();
    if (lane < s) {
        sc->ritz[rank[lane]] = d[lane];
        for (int c = 0; c < s; ++c) {
            double acc = 0.0;
            for (int j = 0; j < s; ++j) acc += Qh[lane * s + j] * A[j + s * c];
            sc->U[lane + s * rank[c]] = acc;
        }
    }
    __syncthreads();
    if (lane < nb) {
        double acc = 0.0;
        for (int j = 0; j < s; ++j) acc += sc->T[(s + lane) * kTld + j] * sc->U[j];
        red[lane] = acc * acc;
    }
    __syncthreads();
    if (lane == 0) {
        double r2 = 0.0;
        for (int q = 0; q < nb; ++q) r2 += red[q];
        double nrm = 0.0;
        for (int i = 0; i < s; ++i) nrm = fmax(nrm, fabs(sc->ritz[i]));
        sc->lam = sc->ritz[0];
        sc->gap = s > 1 ? sc->ritz[1] - sc->ritz[0] : 0.0;
        sc->resid_est = sqrt(r2);
        sc->normT = fmax(sc->normT, nrm);
    }
}

hipError_t launch_block_ritz(const WsLayout &L, void *ws, int s, int nb, hipStream_t st)
{
    if (s < 1 || s > kMaxKrylov || nb < 1 || nb > kMaxBlock || s + nb > kBasisCols) return hipErrorInvalidValue;
    k_block_ritz<<<1, 64, 0, st>>>(ws_ptr<WsScalars>(ws, L.off_scal), s, nb);
    return hipGetLastError();
}

// Thick restart from the Ritz pairs of k_block_ritz: Vnew = [Vold Y_k, Vold[:, s:s+nb)],
// T = [[Theta_k, E^T], [E, 0]] with E = T[s:s+nb, 0:s] Y_k.
__global__ __launch_bounds__(kVecThreads) void k_block_restart(WsScalars *sc, const double *Vold, double *Vnew,
                                                              const double *Iold, double *Inew, int64_t ldv,
                                                              int s, int k, int nb)
{
    __shared__ double Ys[kMaxKrylov * kMaxKrylov];
    __shared__ double Es[kMaxBlock * kMaxKrylov];
    for (int idx = threadIdx.x; idx < s * k; idx += kVecThreads) Ys[idx] = sc->U[idx];
    __syncthreads();
    for (int idx = threadIdx.x; idx < nb * k; idx += kVecThreads) {
        const int r = idx / k, c = idx - r * k;
        double acc = 0.0;
        for (int dd = 0; dd < s; ++dd) acc += sc->T[(s + r) * kTld + dd] * Ys[dd + s * c];
        Es[idx] = acc;
    }
    for (int64_t i = threadIdx.x; i < ldv; i += kVecThreads) {
        for (int c = 0; c < k; ++c) {
            double acc = 0.0, acci = 0.0;
            for (int dd = 0; dd < s; ++dd) {
                acc += Vold[(int64_t)dd * ldv + i] * Ys[dd + s * c];
                acci += Iold[(int64_t)dd * ldv + i] * Ys[dd + s * c];
            }
            Vnew[(int64_t)c * ldv + i] = acc;
            Inew[(int64_t)c * ldv + i] = acci;
        }
        for (int r = 0; r < nb; ++r) Vnew[(int64_t)(k + r) * ldv + i] = Vold[(int64_t)(s + r) * ldv + i];
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < kTld * kTld; idx += kVecThreads) sc->T[idx] = 0.0;
    __syncthreads();
    if (threadIdx.x < k) sc->T[threadIdx.x * kTld + threadIdx.x] = sc->ritz[threadIdx.x];
    for (int idx = threadIdx.x; idx < nb * k; idx += kVecThreads) {
        const int r = idx / k, c = idx - r * k;
        sc->T[(k + r) * kTld + c] = Es[idx];
        sc->T[c * kTld + k + r] = Es[idx];
    }
}

hipError_t launch_block_restart(const WsLayout &L, void *ws, const double *Vold, double *Vnew,
                                const double *Iold, double *Inew, int s, int k, int nb, hipStream_t st)
{
    if (s < 1 || s > kMaxKrylov || k < 1 || k >= s || nb < 1 || nb > kMaxBlock || s + nb > kBasisCols)
        return hipErrorInvalidValue;
    k_block_restart<<<1, kVecThreads, 0, st>>>(ws_ptr<WsScalars>(ws, L.off_scal), Vold, Vnew, Iold, Inew, L.ldv,
                                               s, k, nb);
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
        sc->restarts = 0;
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
    lanczos_step_body(mb.yH, mb.yS, mb.grad, nullptr, mb.sc, mb.kry[cur], mb.img[cur], mb.ld, mb.ncols, j, mode,
                      split, seed);
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
    restart_basis_body(mb.sc, mb.kry[cur], mb.kry[1 - cur], mb.img[cur], mb.img[1 - cur], mb.ld, mb.ncols, m,
                       k, mode, seed);
}

__global__ __launch_bounds__(kVecThreads) void k_ritz_vector_grouped(
    const Member *__restrict__ M, const WorkItem *__restrict__ items, int cur, int m)
{
    const Member &mb = M[items[blockIdx.x].m];
    ritz_vector_body(mb.sc, mb.kry[cur], mb.img[cur], mb.ld, m, mb.y, mb.hy);
}

__global__ __launch_bounds__(kVecThreads) void k_residual_grouped(
    const Member *__restrict__ M, const WorkItem *__restrict__ items, int mode)
{
    const Member &mb = M[items[blockIdx.x].m];
    residual_image_body(mb.sc, mb.y, mb.hy, mb.r, mb.ld, mode);
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
    case kGrpResidual: k_residual_grouped<<<nitems, kVecThreads, 0, st>>>(M, items, i0); break;
    case kGrpUpdate: k_update_grouped<<<nitems, 256, 0, st>>>(M, items); break;
    case kGrpGather: k_gather_scalars<<<nitems, 64, 0, st>>>(M, items, out); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace irl
