// Sampled (variational Monte Carlo) estimators on the determinant set.
//
// Sampling (Methods, "Autoregressive Modeling and Physical Constraints", Eqs.
// autoregressive_factorization and constraint): exact draws from |psi|^2 / Z
// restricted to the fixed-(N_up, N_down) set.  Drawing the spin-orbitals one at
// a time from exact conditionals with one uniform number per sample is the
// inverse transform of the cumulative distribution in ascending key order, so
// the kernels scan |psi|^2 once and binary-search each sample.  The scan runs
// in 64-bit fixed point (psi^2 * 2^k rounded, k chosen so the total stays below
// 2^62): integer sums are exact, so the distribution is monotone and identical
// for any launch shape, and a determinant with psi = 0 is never drawn.
//
// Estimators (Methods, "From SR to a Stable Eigenvalue Problem", Eq.
// centered_hamiltonian; "Practical Matrix-Free Implementation", Eq.
// matrix_vec_prod): with c_r draws of row r out of N, O(x) = D~[x, :] / psi(x)
// and E_loc(x) = (H psi)(x) / psi(x), every sample mean over the draws is a
// weighted sum over rows with q_r = Z c_r / (N psi_r^2):
//   E = (1/N) sum_r c_r E_loc,r
//   F = (2/Z) D~^T (q (H psi - E psi))
//   (y_H, y_S) = (D~^T (q E_loc w), D~^T (q w)),  w = D~ v,
// so that (y_H - E y_S) / Z is the sample mean of O (E_loc - E) (O . v).

#include "internal.h"

namespace irl {

namespace {

constexpr int kScanThreads = 1024;
constexpr int kScanWaves = kScanThreads / kWave;
constexpr int kScanPer = 8;                          // consecutive rows per thread
constexpr int64_t kScanChunk = (int64_t)kScanThreads * kScanPer;
constexpr int kVmcThreads = 256;
constexpr int kVmcBlocks = 1024;                     // row blocks of the weight passes

__device__ __forceinline__ uint64_t fixed_weight(double p, int k)
{
    return (uint64_t)rint(ldexp(p * p, k));
}

// values scanned: the fixed-point weight of a row, or whether it was drawn
struct WeightVal {
    const double *psi;
    int k;
    __device__ uint64_t operator()(int64_t i) const { return fixed_weight(psi[i], k); }
};
struct DrawnVal {
    const uint32_t *counts;
    __device__ uint64_t operator()(int64_t i) const { return counts[i] ? 1ull : 0ull; }
};

// this thread's values and their sum
template <typename F>
__device__ __forceinline__ uint64_t thread_values(const F &f, int64_t ns, int64_t base, uint64_t *w)
{
    uint64_t s = 0;
#pragma unroll
    for (int e = 0; e < kScanPer; ++e) {
        const int64_t i = base + e;
        w[e] = i < ns ? f(i) : 0ull;
        s += w[e];
    }
    return s;
}

// exclusive prefix of v over the block's threads and the block total (integer: exact)
__device__ uint64_t block_exclusive(uint64_t v, uint64_t *sh, uint64_t *total)
{
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
    uint64_t x = v;
    for (int off = 1; off < kWave; off <<= 1) {
        const uint64_t y = __shfl_up(x, off, kWave);
        if (lane >= off) x += y;
    }
    if (lane == kWave - 1) sh[wv] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t acc = 0;
        for (int i = 0; i < kScanWaves; ++i) {
            const uint64_t t = sh[i];
            sh[i] = acc;
            acc += t;
        }
        sh[kScanWaves] = acc;
    }
    __syncthreads();
    *total = sh[kScanWaves];
    return sh[wv] + (x - v);
}

template <typename F>
__global__ __launch_bounds__(kScanThreads) void k_scan_chunks(F f, int64_t ns, uint64_t *__restrict__ tot)
{
    __shared__ uint64_t sh[kScanWaves + 1];
    uint64_t w[kScanPer];
    const int64_t base = (int64_t)blockIdx.x * kScanChunk + (int64_t)threadIdx.x * kScanPer;
    uint64_t total;
    block_exclusive(thread_values(f, ns, base, w), sh, &total);
    if (threadIdx.x == 0) tot[blockIdx.x] = total;
}

// exclusive offsets of the chunk totals, in place; the grand total into tot[nc]
__global__ __launch_bounds__(kScanThreads) void k_scan_offsets(uint64_t *__restrict__ tot, int64_t nc)
{
    __shared__ uint64_t sh[kScanWaves + 1];
    uint64_t carry = 0;
    for (int64_t b = 0; b < nc; b += kScanThreads) {
        const int64_t i = b + threadIdx.x;
        const uint64_t v = i < nc ? tot[i] : 0ull;
        uint64_t seg;
        const uint64_t ex = block_exclusive(v, sh, &seg);
        if (i < nc) tot[i] = carry + ex;
        carry += seg;
        __syncthreads();
    }
    if (threadIdx.x == 0) tot[nc] = carry;
}

template <typename F>
__global__ __launch_bounds__(kScanThreads) void k_scan_apply(F f, int64_t ns, const uint64_t *__restrict__ off,
                                                            uint64_t *__restrict__ cum)
{
    __shared__ uint64_t sh[kScanWaves + 1];
    uint64_t w[kScanPer];
    const int64_t base = (int64_t)blockIdx.x * kScanChunk + (int64_t)threadIdx.x * kScanPer;
    uint64_t total;
    uint64_t acc = off[blockIdx.x] + block_exclusive(thread_values(f, ns, base, w), sh, &total);
#pragma unroll
    for (int e = 0; e < kScanPer; ++e) {
        acc += w[e];
        if (base + e < ns) cum[base + e] = acc;
    }
}

// sample s: the first row whose cumulative weight exceeds floor(u_s T); u outside
// [0, 1) (or NaN) is clamped into it
__global__ __launch_bounds__(kVmcThreads) void k_vmc_draw(const double *__restrict__ u, int64_t nsamp,
                                                         const uint64_t *__restrict__ cum, int64_t ns,
                                                         const uint64_t *__restrict__ totp,
                                                         uint32_t *__restrict__ counts, int64_t *__restrict__ rows)
{
    const int64_t s = (int64_t)blockIdx.x * kVmcThreads + threadIdx.x;
    if (s >= nsamp) return;
    const uint64_t T = *totp;
    const double x = u[s] * (double)T;
    uint64_t t = 0;
    if (x > 0.0) t = x < (double)T ? (uint64_t)x : T - 1;
    if (t >= T) t = T - 1;
    int64_t lo = 0, hi = ns - 1;
    while (lo < hi) {
        const int64_t mid = lo + ((hi - lo) >> 1);
        if (cum[mid] > t)
            hi = mid;
        else
            lo = mid + 1;
    }
    atomicAdd(&counts[lo], 1u);
    if (rows) rows[s] = lo;
}

__global__ void k_fill_u32(uint32_t *p, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

// fixed-order sum over a 256-thread block; result valid in thread 0
__device__ double block_sum256(double v, double *sh)
{
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, kWave);
    if (lane == 0) sh[wv] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < kVmcThreads / kWave; ++i) s += sh[i];
    __syncthreads();
    return s;
}

// q_r = Z c_r / (N psi_r^2); per-block sums of c_r E_loc,r and of the distinct rows
__global__ __launch_bounds__(kVmcThreads) void k_vmc_weights(const uint32_t *__restrict__ counts,
                                                            const double *__restrict__ psi,
                                                            const double *__restrict__ hpsi, int64_t ns,
                                                            double zn, double *__restrict__ q,
                                                            double *__restrict__ part)
{
    __shared__ double sh[kVmcThreads / kWave];
    double se = 0.0, su = 0.0;
    for (int64_t r = (int64_t)blockIdx.x * kVmcThreads + threadIdx.x; r < ns;
         r += (int64_t)gridDim.x * kVmcThreads) {
        const uint32_t c = counts[r];
        double qr = 0.0;
        if (c) {
            const double p = psi[r];
            qr = zn * (double)c / (p * p);
            se += (double)c * (hpsi[r] / p);
            su += 1.0;
        }
        q[r] = qr;
    }
    const double a = block_sum256(se, sh);
    const double b = block_sum256(su, sh);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = a;
        part[2 * blockIdx.x + 1] = b;
    }
}

// fixed-order sum of n <= kVmcBlocks partials (stride `stride`) over one
// 1024-thread block; result valid in thread 0
__device__ double partial_sum(const double *__restrict__ part, int n, int stride, double *sh)
{
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
    double v = (int)threadIdx.x < n ? part[(int64_t)threadIdx.x * stride] : 0.0;
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, kWave);
    if (lane == 0) sh[wv] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < kVmcBlocks / kWave; ++i) s += sh[i];
    __syncthreads();
    return s;
}

// E = sum / N into sc->E_el and out[0]; distinct rows into out[1]
__global__ __launch_bounds__(kVmcBlocks) void k_vmc_energy(const double *__restrict__ part, int nblk, double inv_n,
                                                          WsScalars *sc, double *out)
{
    __shared__ double sh[kVmcBlocks / kWave];
    const double e = partial_sum(part, nblk, 2, sh);
    const double un = partial_sum(part + 1, nblk, 2, sh);
    if (threadIdx.x == 0) {
        sc->E_el = e * inv_n;
        out[0] = e * inv_n;
        out[1] = un;
    }
}

// right-hand side of the sampled gradient, y_r = q_r (H psi - E psi)_r, and
// per-block sums of c_r (E_loc,r - E)^2
__global__ __launch_bounds__(kVmcThreads) void k_vmc_rhs(const uint32_t *__restrict__ counts,
                                                        const double *__restrict__ psi,
                                                        const double *__restrict__ hpsi,
                                                        const double *__restrict__ q, int64_t ns,
                                                        const WsScalars *sc, double *__restrict__ y,
                                                        double *__restrict__ part)
{
    __shared__ double sh[kVmcThreads / kWave];
    const double E = sc->E_el;
    double sv = 0.0;
    for (int64_t r = (int64_t)blockIdx.x * kVmcThreads + threadIdx.x; r < ns;
         r += (int64_t)gridDim.x * kVmcThreads) {
        const double qr = q[r];
        double yr = 0.0;
        if (qr != 0.0) {
            const double p = psi[r], h = hpsi[r];
            yr = qr * (h - E * p);
            const double d = h / p - E;
            sv += (double)counts[r] * d * d;
        }
        y[r] = yr;
    }
    const double a = block_sum256(sv, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = a;
}

__global__ __launch_bounds__(kVmcBlocks) void k_vmc_variance(const double *__restrict__ part, int nblk,
                                                            double inv_n, double *out)
{
    __shared__ double sh[kVmcBlocks / kWave];
    const double v = partial_sum(part, nblk, 1, sh);
    if (threadIdx.x == 0) out[2] = v * inv_n;
}

// gradient right-hand side on the gathered rows: y_j = q_j psi_j (E_loc,j - E)
__global__ __launch_bounds__(kVmcThreads) void k_vmc_rhs_rows(const double *__restrict__ cq,
                                                             const double *__restrict__ cpsi,
                                                             const double *__restrict__ cel, int64_t nrows,
                                                             const WsScalars *sc, double *__restrict__ y)
{
    const double E = sc->E_el;
    for (int64_t j = (int64_t)blockIdx.x * kVmcThreads + threadIdx.x; j < nrows;
         j += (int64_t)gridDim.x * kVmcThreads)
        y[j] = cq[j] * cpsi[j] * (cel[j] - E);
}

// the sampled operator's diagonal: w <- q w, u <- q E_loc w (nb columns of ns)
__global__ __launch_bounds__(kVmcThreads) void k_vmc_diag(const double *__restrict__ q,
                                                         const double *__restrict__ psi,
                                                         const double *__restrict__ hpsi, int64_t ns, int nb,
                                                         double *__restrict__ w, double *__restrict__ u)
{
    for (int64_t r = (int64_t)blockIdx.x * kVmcThreads + threadIdx.x; r < ns;
         r += (int64_t)gridDim.x * kVmcThreads) {
        const double qr = q[r];
        const double el = qr != 0.0 ? hpsi[r] / psi[r] : 0.0;
        for (int c = 0; c < nb; ++c) {
            const double x = qr * w[(int64_t)c * ns + r];
            w[(int64_t)c * ns + r] = x;
            u[(int64_t)c * ns + r] = x * el;
        }
    }
}

// compact slot of each drawn row: crow[cum_r - 1] = r (cum inclusive over drawn flags)
__global__ __launch_bounds__(kVmcThreads) void k_vmc_index(const uint32_t *__restrict__ counts,
                                                          const uint64_t *__restrict__ cum, int64_t ns,
                                                          int64_t *__restrict__ crow)
{
    for (int64_t r = (int64_t)blockIdx.x * kVmcThreads + threadIdx.x; r < ns;
         r += (int64_t)gridDim.x * kVmcThreads)
        if (counts[r]) crow[cum[r] - 1] = r;
}

// one wavefront per drawn row j < *nup: key, psi, weight, local energy and the d row
__global__ __launch_bounds__(kVmcThreads) void k_vmc_gather(const int64_t *__restrict__ crow,
                                                           const uint64_t *__restrict__ nup, int64_t slots,
                                                           const uint64_t *__restrict__ keys,
                                                           const double *__restrict__ psi,
                                                           const double *__restrict__ hpsi,
                                                           const double *__restrict__ q,
                                                           const double *__restrict__ dfac, int hfac,
                                                           uint64_t *__restrict__ ckeys, double *__restrict__ cpsi,
                                                           double *__restrict__ cq, double *__restrict__ cel,
                                                           double *__restrict__ cfac)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t nu = (int64_t)*nup;
    const int64_t waves = (int64_t)gridDim.x * (kVmcThreads / kWave);
    for (int64_t j = (int64_t)blockIdx.x * (kVmcThreads / kWave) + threadIdx.x / kWave; j < nu && j < slots;
         j += waves) {
        const int64_t r = crow[j];
        if (lane == 0) {
            ckeys[j] = keys[r];
            cpsi[j] = psi[r];
            cq[j] = q[r];
            cel[j] = hpsi[r] / psi[r];
        }
        for (int h = lane; h < hfac; h += kWave) cfac[j * hfac + h] = dfac[r * hfac + h];
    }
}

// the sampled operator's diagonal on gathered rows: w <- q w, u <- q E_loc w
__global__ __launch_bounds__(kVmcThreads) void k_vmc_diag_rows(const double *__restrict__ cq,
                                                              const double *__restrict__ cel, int64_t nrows,
                                                              double *__restrict__ w, double *__restrict__ u)
{
    for (int64_t j = (int64_t)blockIdx.x * kVmcThreads + threadIdx.x; j < nrows;
         j += (int64_t)gridDim.x * kVmcThreads) {
        const double x = cq[j] * w[j];
        w[j] = x;
        u[j] = x * cel[j];
    }
}

unsigned row_blocks(int64_t ns)
{
    const int64_t b = (ns + kVmcThreads - 1) / kVmcThreads;
    return (unsigned)(b < kVmcBlocks ? (b > 0 ? b : 1) : kVmcBlocks);
}

}  // namespace

int64_t vmc_scan_chunks(int64_t ns)
{
    return (ns + kScanChunk - 1) / kScanChunk;
}

int vmc_weight_blocks(int64_t ns)
{
    return (int)row_blocks(ns);
}

hipError_t launch_vmc_sample(const WsLayout &L, void *ws, const double *u, int64_t nsamp, int k, double Z,
                             int64_t *rows, double *out, hipStream_t st)
{
    const int64_t ns = L.ns;
    const double *psi = ws_ptr<double>(ws, L.off_psi), *hpsi = ws_ptr<double>(ws, L.off_hpsi);
    uint64_t *cum = ws_ptr<uint64_t>(ws, L.off_w);
    uint32_t *counts = ws_ptr<uint32_t>(ws, L.off_u);
    uint64_t *tot = ws_ptr<uint64_t>(ws, L.off_part);
    double *part = ws_ptr<double>(ws, L.off_red);
    double *q = ws_ptr<double>(ws, L.off_q);
    double *y = ws_ptr<double>(ws, L.off_w);       // after the draws the scan is no longer needed
    WsScalars *sc = ws_ptr<WsScalars>(ws, L.off_scal);
    const int64_t nc = vmc_scan_chunks(ns);
    const unsigned nb = row_blocks(ns);
    const WeightVal wv{psi, k};
    k_scan_chunks<<<(unsigned)nc, kScanThreads, 0, st>>>(wv, ns, tot);
    k_scan_offsets<<<1, kScanThreads, 0, st>>>(tot, nc);
    k_scan_apply<<<(unsigned)nc, kScanThreads, 0, st>>>(wv, ns, tot, cum);
    k_fill_u32<<<nb, kVmcThreads, 0, st>>>(counts, ns);
    k_vmc_draw<<<(unsigned)((nsamp + kVmcThreads - 1) / kVmcThreads), kVmcThreads, 0, st>>>(
        u, nsamp, cum, ns, tot + nc, counts, rows);
    const double inv_n = 1.0 / (double)nsamp;
    k_vmc_weights<<<nb, kVmcThreads, 0, st>>>(counts, psi, hpsi, ns, Z * inv_n, q, part);
    k_vmc_energy<<<1, kVmcBlocks, 0, st>>>(part, (int)nb, inv_n, sc, out);
    k_vmc_rhs<<<nb, kVmcThreads, 0, st>>>(counts, psi, hpsi, q, ns, sc, y, part);
    k_vmc_variance<<<1, kVmcBlocks, 0, st>>>(part, (int)nb, inv_n, out);
    return hipGetLastError();
}

hipError_t launch_vmc_gather(const WsLayout &L, void *ws, const uint64_t *keys, int hfac, hipStream_t st)
{
    const int64_t ns = L.ns;
    const uint32_t *counts = ws_ptr<uint32_t>(ws, L.off_u);
    uint64_t *cum = ws_ptr<uint64_t>(ws, L.off_w);
    uint64_t *tot = ws_ptr<uint64_t>(ws, L.off_part);
    const int64_t nc = vmc_scan_chunks(ns);
    const DrawnVal dv{counts};
    k_scan_chunks<<<(unsigned)nc, kScanThreads, 0, st>>>(dv, ns, tot);
    k_scan_offsets<<<1, kScanThreads, 0, st>>>(tot, nc);
    k_scan_apply<<<(unsigned)nc, kScanThreads, 0, st>>>(dv, ns, tot, cum);
    int64_t *crow = ws_ptr<int64_t>(ws, L.off_crow);
    k_vmc_index<<<row_blocks(ns), kVmcThreads, 0, st>>>(counts, cum, ns, crow);
    const int64_t waves_per_block = kVmcThreads / kWave;
    int64_t blocks = (ns + waves_per_block - 1) / waves_per_block;
    if (blocks > 16384) blocks = 16384;
    k_vmc_gather<<<(unsigned)blocks, kVmcThreads, 0, st>>>(
        crow, tot + nc, ns, keys, ws_ptr<double>(ws, L.off_psi), ws_ptr<double>(ws, L.off_hpsi),
        ws_ptr<double>(ws, L.off_q), ws_ptr<double>(ws, L.off_fac), hfac, ws_ptr<uint64_t>(ws, L.off_ckeys),
        ws_ptr<double>(ws, L.off_cpsi), ws_ptr<double>(ws, L.off_cq), ws_ptr<double>(ws, L.off_cel),
        ws_ptr<double>(ws, L.off_cfac));
    return hipGetLastError();
}

hipError_t launch_vmc_rhs_rows(const WsLayout &L, void *ws, int64_t nrows, double *y, hipStream_t st)
{
    k_vmc_rhs_rows<<<row_blocks(nrows), kVmcThreads, 0, st>>>(
        ws_ptr<double>(ws, L.off_cq), ws_ptr<double>(ws, L.off_cpsi), ws_ptr<double>(ws, L.off_cel), nrows,
        ws_ptr<WsScalars>(ws, L.off_scal), y);
    return hipGetLastError();
}

hipError_t launch_vmc_diag_rows(const WsLayout &L, void *ws, int64_t nrows, double *w, double *u, hipStream_t st)
{
    k_vmc_diag_rows<<<row_blocks(nrows), kVmcThreads, 0, st>>>(ws_ptr<double>(ws, L.off_cq),
                                                               ws_ptr<double>(ws, L.off_cel), nrows, w, u);
    return hipGetLastError();
}

hipError_t launch_vmc_diag(const WsLayout &L, void *ws, double *w, double *u, int nb, hipStream_t st)
{
    k_vmc_diag<<<row_blocks(L.ns), kVmcThreads, 0, st>>>(ws_ptr<double>(ws, L.off_q), ws_ptr<double>(ws, L.off_psi),
                                                         ws_ptr<double>(ws, L.off_hpsi), L.ns, nb, w, u);
    return hipGetLastError();
}

}  // namespace irl
