// Network amplitude and Jacobian rows of D~ = [psi, d psi / d theta] on gfx950.
//
// Tangent basis of the linearised wavefunction (Methods, "From SR to a Stable
// Eigenvalue Problem"): chi_0 = psi, chi_i = d psi / d theta_i.  Network
// (one hidden tanh layer, real):
//   x_v = occupation of spin-orbital v, t_h = tanh(b_h + sum_v W_hv x_v),
//   psi = sum_v a_v x_v + sum_h t_h,
//   d psi/d a_v = x_v, d psi/d b_h = 1 - t_h^2, d psi/d W_hv = (1 - t_h^2) x_v.
// One wavefront per determinant: lanes own hidden units for the forward pass,
// then the whole row (P + 1 values plus zero padding) is written with
// coalesced non-temporal stores (HBM-write bound: D~ is written once per step).
#include "internal.h"

namespace irl {

constexpr int kMaxHidden = 1024;

// Row write of D~ = [psi, x, 1 - t^2, (1 - t^2) (x) x]: each lane owns CPL
// consecutive columns per pass, so every store instruction of the wave covers
// 64 * 16 contiguous bytes (CPL = 2: FP64 copy, plus the FP32 copy when present;
// CPL = 4: FP32 copy only).  Inside the W block (column 1 + V + H + h V + v) the
// lane tracks (h, v) incrementally.
template <int CPL>
__device__ __forceinline__ void write_row(uint64_t xm, int64_t row, int V, int H, double psi,
                                          const double *dsh, double *__restrict__ D64, int64_t ld64,
                                          float *__restrict__ D32, int64_t ld32, int lane)
{
    const int64_t P1 = (int64_t)V * H + H + V + 1;
    const int baseW = V + H + 1;
    const int64_t ldw = D64 ? ld64 : ld32;
    constexpr int kStep = CPL * kWave;
    const int qh = kStep / V, rv = kStep - qh * V;   // (h, v) advance per pass
    int64_t c0 = CPL * lane;
    int hh = 0, vv = 0;
    if (c0 >= baseW) {
        const int idx = (int)(c0 - baseW);
        hh = idx / V;
        vv = idx - hh * V;
    }
    for (; c0 < ldw; c0 += kStep) {
        double val[CPL];
        if (c0 >= baseW && c0 + CPL - 1 < P1) {
            int h2 = hh, v2 = vv;
#pragma unroll
            for (int q = 0; q < CPL; ++q) {
                val[q] = ((xm >> v2) & 1ull) ? dsh[h2] : 0.0;
                if (++v2 == V) {
                    v2 = 0;
                    ++h2;
                }
            }
        } else {
#pragma unroll
            for (int q = 0; q < CPL; ++q) {
                const int64_t c = c0 + q;
                double x;
                if (c == 0) {
                    x = psi;
                } else if (c <= V) {
                    x = (double)((xm >> (c - 1)) & 1ull);
                } else if (c < baseW) {
                    x = dsh[c - V - 1];
                } else if (c < P1) {
                    const int idx = (int)(c - baseW);
                    const int h2 = idx / V;
                    x = ((xm >> (idx - h2 * V)) & 1ull) ? dsh[h2] : 0.0;
                } else {
                    x = 0.0;
                }
                val[q] = x;
            }
        }
        // (h, v) of the next pass's first column
        if (c0 + kStep >= baseW) {
            if (c0 < baseW) {
                const int idx = (int)(c0 + kStep - baseW);
                hh = idx / V;
                vv = idx - hh * V;
            } else {
                hh += qh;
                vv += rv;
                if (vv >= V) {
                    vv -= V;
                    ++hh;
                }
            }
        }
        if constexpr (CPL == 2) {
            typedef double d2 __attribute__((ext_vector_type(2)));
            typedef float f2 __attribute__((ext_vector_type(2)));
            d2 a = {val[0], val[1]};
            __builtin_nontemporal_store(a, (d2 *)(D64 + row * ld64 + c0));
            if (D32) {
                f2 b2 = {(float)val[0], (float)val[1]};
                __builtin_nontemporal_store(b2, (f2 *)(D32 + row * ld32 + c0));
            }
        } else {
            typedef float f4 __attribute__((ext_vector_type(4)));
            f4 v4 = {(float)val[0], (float)val[1], (float)val[2], (float)val[3]};
            __builtin_nontemporal_store(v4, (f4 *)(D32 + row * ld32 + c0));
        }
    }
}

// one determinant row on one wavefront (dsh: the wave's H-long scratch in LDS)
__device__ __forceinline__ void nqs_row(uint64_t key, int64_t row, int n, int V, int H,
                                        const double *__restrict__ theta, double *__restrict__ D64,
                                        int64_t ld64, float *__restrict__ D32, int64_t ld32,
                                        double *__restrict__ psi_out, double *__restrict__ dfac,
                                        double *dsh, int lane)
{
    const double *a = theta, *b = theta + V, *W = theta + V + H;
    // x as a bit mask over v: alpha orbitals at v < n, beta at v = n + p
    uint64_t xm = (key & 0xffffffffull) | ((key >> 32) << n);
    double tsum = 0.0;
    for (int h = lane; h < H; h += kWave) {
        double z = b[h];
        for (uint64_t m = xm; m; m &= m - 1) z += W[(size_t)h * V + (__ffsll((unsigned long long)m) - 1)];
        double t = tanh(z);
        tsum += t;
        dsh[h] = 1.0 - t * t;
        if (dfac) dfac[row * H + h] = 1.0 - t * t;
    }
    double asum = 0.0;
    if (lane == 0)
        for (uint64_t m = xm; m; m &= m - 1) asum += a[__ffsll((unsigned long long)m) - 1];
    // butterfly: every lane ends with the same (bitwise) total
    for (int off = 32; off > 0; off >>= 1) tsum += __shfl_xor(tsum, off, kWave);
    const double psi = __shfl(asum, 0, kWave) + tsum;
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (lane == 0) psi_out[row] = psi;
    if (D64)
        write_row<2>(xm, row, V, H, psi, dsh, D64, ld64, D32, ld32, lane);
    else if (D32)
        write_row<4>(xm, row, V, H, psi, dsh, nullptr, ld64, D32, ld32, lane);
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__global__ __launch_bounds__(256) void k_nqs_dtilde(const uint64_t *__restrict__ keys, int64_t ns,
                                                    int n, int V, int H,
                                                    const double *__restrict__ theta,
                                                    double *__restrict__ D64, int64_t ld64,
                                                    float *__restrict__ D32, int64_t ld32,
                                                    double *__restrict__ psi_out,
                                                    double *__restrict__ dfac)
{
    __shared__ double dsh[4][kMaxHidden];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t nwaves = (int64_t)gridDim.x * 4;
    for (int64_t row = (int64_t)blockIdx.x * 4 + wv; row < ns; row += nwaves)
        nqs_row(keys[row], row, n, V, H, theta, D64, ld64, D32, ld32, psi_out, dfac, dsh[wv], lane);
}

// grouped: item = rows [r0, r1) of member m, interleaved over the 4 waves
__global__ __launch_bounds__(256) void k_nqs_dtilde_grouped(const Member *__restrict__ M,
                                                            const WorkItem *__restrict__ items,
                                                            int n)
{
    __shared__ double dsh[4][kMaxHidden];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const WorkItem it = items[blockIdx.x];
    const Member &mb = M[it.m];
    for (int64_t row = it.r0 + wv; row < it.r1; row += 4)
        nqs_row(mb.ham.keys[row], row, mb.ham.n, mb.V, mb.H, mb.theta, const_cast<double *>(mb.D64),
                mb.ld, const_cast<float *>(mb.D32), mb.ld, mb.psi, nullptr, dsh[wv], lane);
}

hipError_t launch_nqs_dtilde_grouped(const Member *M, const WorkItem *items, int nitems, int n,
                                     uint32_t flags, hipStream_t st)
{
    (void)n;
    (void)flags;
    if (nitems <= 0) return hipSuccess;
    k_nqs_dtilde_grouped<<<nitems, 256, 0, st>>>(M, items, 0);
    return hipGetLastError();
}

hipError_t launch_nqs_dtilde(const irl_system *s, int V, int H, const double *theta,
                             const WsLayout &L, void *ws, hipStream_t st)
{
    double *D64 = (L.flags & IRL_WS_FP64) ? ws_ptr<double>(ws, L.off_d64) : nullptr;
    float *D32 = (L.flags & IRL_WS_FP32) ? ws_ptr<float>(ws, L.off_d32) : nullptr;
    if (!D64 && !D32 && (L.flags & IRL_WS_FACTORED)) return launch_fac_forward(s, L, ws, theta, st);
    int64_t blocks = (L.ns + 3) / 4;
    if (blocks > 16384) blocks = 16384;
    double *dfac = (L.flags & IRL_WS_FACTORED) ? ws_ptr<double>(ws, L.off_fac) : nullptr;
    k_nqs_dtilde<<<(unsigned)blocks, 256, 0, st>>>(s->d.keys, L.ns, s->n, V, H, theta, D64,
                                                   L.ld64, D32, L.ld32,
                                                   ws_ptr<double>(ws, L.off_psi), dfac);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// FP64 gradient without an FP64 copy of D~ (Methods, "From SR to a Stable
// Eigenvalue Problem": the energy gradient is the Jacobian transposed applied to
// the local-energy residual).  With c_x = (H psi)_x - E psi_x, the entries of
// D~^T c are, per column block of D~:
//   psi column:   sum_x c_x psi_x
//   a_v:          sum_x c_x x_v
//   b_h:          sum_x c_x (1 - t_xh^2)
//   W_hv:         sum_x c_x (1 - t_xh^2) x_v
// recomputed from theta in FP64 (the network pass costs far less than a D~
// stream).  Grid (hidden tiles of 64, row blocks): lane = hidden unit of the
// tile, W rows of the tile in LDS; every row's occupation mask is uniform over
// the wave, so the W_h. accumulators are updated with a static loop over v.
// The 4 waves are combined in a fixed order and wave 0 writes the block's
// partial row into the second half of part (the first half is zeroed), the
// layout the two-level D~^T reduction reads.
constexpr int kGradVmax = 64;

// D~^T c over rows [r0, r1) for the hidden units of tile ht, c_r = y_r - coef psi_r,
// with d = 1 - t^2 recomputed from theta (W rows of the tile staged in LDS).  VMAX
// >= V bounds the static loop over the visible units.  The 4 waves are combined in
// a fixed order and wave 0 writes entries [0, ldv) of the partial row `out` that
// belong to this tile (tile 0 also writes the psi, x and padding entries).
template <int VMAX>
__device__ __forceinline__ void vjp_block(const uint64_t *__restrict__ keys, int64_t r0, int64_t r1,
                                          int n, int V, int H, int ht, const double *__restrict__ theta,
                                          const double *__restrict__ psi, const double *__restrict__ y,
                                          double coef, double *__restrict__ out, int64_t ldv, double *Wt,
                                          double *red)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int h = ht * 64 + lane;
    const bool hv = h < H;
    constexpr int kWs = kGradVmax + 1;   // odd LDS row stride: lanes read distinct banks
    const double *b = theta + V, *W = theta + V + H;
    for (int i = threadIdx.x; i < 64 * kWs; i += blockDim.x) {
        const int hh = i / kWs, v = i - hh * kWs;
        Wt[i] = (v < V && ht * 64 + hh < H) ? W[(size_t)(ht * 64 + hh) * V + v] : 0.0;
    }
    __syncthreads();
    const double bh = hv ? b[h] : 0.0;
    double accW[VMAX];
#pragma unroll
    for (int v = 0; v < VMAX; ++v) accW[v] = 0.0;
    double accB = 0.0, accA = 0.0, acc0 = 0.0;
    auto row_d = [&](uint64_t xm) -> double {
        double z = bh;
        for (uint64_t m = xm; m; m &= m - 1) z += Wt[lane * kWs + (__ffsll((unsigned long long)m) - 1)];
        const double t = tanh(z);
        return 1.0 - t * t;
    };
    auto accumulate = [&](double c, double dh, double ps, uint64_t xm) {
        const double d = c * dh;
        accB += d;
#pragma unroll
        for (int v = 0; v < VMAX; ++v) accW[v] += ((xm >> v) & 1ull) ? d : 0.0;
        if (ht == 0) {
            accA += ((xm >> lane) & 1ull) ? c : 0.0;
            acc0 += c * ps;
        }
    };
    int64_t r = r0 + wv;
    // two rows per pass: their loads are independent and overlap
    for (; r + 4 < r1; r += 8) {
        const uint64_t k0 = keys[r], k1 = keys[r + 4];
        const uint64_t x0 = (k0 & 0xffffffffull) | ((k0 >> 32) << n);
        const uint64_t x1 = (k1 & 0xffffffffull) | ((k1 >> 32) << n);
        const double p0 = psi[r], p1 = psi[r + 4];
        const double c0 = y[r] - coef * p0, c1 = y[r + 4] - coef * p1;
        const double d0 = row_d(x0), d1 = row_d(x1);
        accumulate(c0, d0, p0, x0);
        accumulate(c1, d1, p1, x1);
    }
    for (; r < r1; r += 4) {
        const uint64_t k0 = keys[r];
        const uint64_t x0 = (k0 & 0xffffffffull) | ((k0 >> 32) << n);
        const double p0 = psi[r];
        accumulate(y[r] - coef * p0, row_d(x0), p0, x0);
    }
    // fixed-order combination of the 4 waves: ((w0 + w1) + w2) + w3
    constexpr int kRs = kGradVmax + 3;
    for (int src = 1; src < 4; ++src) {
        __syncthreads();
        if (wv == src) {
#pragma unroll
            for (int v = 0; v < VMAX; ++v) red[lane * kRs + v] = accW[v];
            red[lane * kRs + kGradVmax] = accB;
            red[lane * kRs + kGradVmax + 1] = accA;
            red[lane * kRs + kGradVmax + 2] = acc0;
        }
        __syncthreads();
        if (wv == 0) {
#pragma unroll
            for (int v = 0; v < VMAX; ++v) accW[v] += red[lane * kRs + v];
            accB += red[lane * kRs + kGradVmax];
            accA += red[lane * kRs + kGradVmax + 1];
            acc0 += red[lane * kRs + kGradVmax + 2];
        }
    }
    if (wv != 0) return;
    const int64_t P1 = (int64_t)V * H + H + V + 1;
    if (hv) {
        out[1 + V + h] = accB;
#pragma unroll
        for (int v = 0; v < VMAX; ++v)
            if (v < V) out[1 + V + H + (int64_t)h * V + v] = accW[v];
    }
    if (ht == 0) {
        if (lane < V) out[1 + lane] = accA;
        if (lane == 0) out[0] = acc0;
        for (int64_t c = P1 + lane; c < ldv; c += 64) out[c] = 0.0;
    }
}

__global__ __launch_bounds__(256) void k_nqs_grad(const uint64_t *__restrict__ keys, int64_t ns, int n,
                                                  int V, int H, const double *__restrict__ theta,
                                                  const double *__restrict__ psi,
                                                  const double *__restrict__ hpsi,
                                                  const WsScalars *__restrict__ sc,
                                                  double *__restrict__ part, int64_t ldv, int nblk)
{
    __shared__ double Wt[64 * (kGradVmax + 1)];
    __shared__ double red[64 * (kGradVmax + 3)];
    const int ht = blockIdx.x, rb = blockIdx.y;
    const int64_t per = (ns + nblk - 1) / nblk;
    const int64_t r0 = (int64_t)rb * per, r1 = min(ns, r0 + per);
    double *pa = part + (int64_t)rb * 2 * ldv;
    // the first half of the partial row (D~^T psi) is not formed here
    if (ht == 0)
        for (int64_t c = threadIdx.x; c < ldv; c += blockDim.x) pa[c] = 0.0;
    vjp_block<kGradVmax>(keys, r0, r1, n, V, H, ht, theta, psi, hpsi, sc->E_el, pa + ldv, ldv, Wt, red);
}


hipError_t launch_nqs_grad(const irl_system *s, int V, int H, const double *theta, const WsLayout &L,
                           void *ws, int nblk, hipStream_t st)
{
    if (V > kGradVmax) return hipErrorInvalidValue;
    const int htiles = (H + 63) / 64;
    k_nqs_grad<<<dim3(htiles, nblk), 256, 0, st>>>(s->d.keys, L.ns, s->n, V, H, theta,
                                                   ws_ptr<double>(ws, L.off_psi),
                                                   ws_ptr<double>(ws, L.off_hpsi),
                                                   ws_ptr<WsScalars>(ws, L.off_scal),
                                                   ws_ptr<double>(ws, L.off_part), L.ldv, nblk);
    return hipGetLastError();
}

// Copy a caller-provided D~ into the workspace copies (zero padding), and
// column 0 into psi.
template <typename TS>
__global__ void k_dtilde_import(const TS *__restrict__ src, int64_t lds, int64_t ncols, int64_t ns,
                                double *D64, int64_t ld64, float *D32, int64_t ld32, double *psi)
{
    const int64_t row = blockIdx.y + (int64_t)blockIdx.z * 65535;
    if (row >= ns) return;
    const int64_t ldw = D64 ? ld64 : ld32;
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < ldw;
         c += (int64_t)gridDim.x * blockDim.x) {
        double x = c < ncols ? (double)src[row * lds + c] : 0.0;
        if (D64) D64[row * ld64 + c] = x;
        if (D32 && c < ld32) D32[row * ld32 + c] = (float)x;
        if (c == 0) psi[row] = x;
    }
}

hipError_t launch_dtilde_import(const void *D, int64_t ld, int64_t ncols, int dtype,
                                const WsLayout &L, void *ws, hipStream_t st)
{
    double *D64 = (L.flags & IRL_WS_FP64) ? ws_ptr<double>(ws, L.off_d64) : nullptr;
    float *D32 = (L.flags & IRL_WS_FP32) ? ws_ptr<float>(ws, L.off_d32) : nullptr;
    double *psi = ws_ptr<double>(ws, L.off_psi);
    int64_t ldw = D64 ? L.ld64 : L.ld32;
    dim3 grid((unsigned)((ldw + 255) / 256 > 64 ? 64 : (ldw + 255) / 256),
              (unsigned)(L.ns < 65535 ? L.ns : 65535), (unsigned)((L.ns + 65534) / 65535));
    if (dtype == IRL_FP64)
        k_dtilde_import<double><<<grid, 256, 0, st>>>((const double *)D, ld, ncols, L.ns, D64,
                                                      L.ld64, D32, L.ld32, psi);
    else
        k_dtilde_import<float><<<grid, 256, 0, st>>>((const float *)D, ld, ncols, L.ns, D64,
                                                     L.ld64, D32, L.ld32, psi);
    return hipGetLastError();
}

}  // namespace irl
