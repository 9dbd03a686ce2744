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

// one determinant row on one wavefront (dsh: the wave's H-long scratch in LDS)
__device__ __forceinline__ void nqs_row(uint64_t key, int64_t row, int n, int V, int H,
                                        const double *__restrict__ theta, double *__restrict__ D64,
                                        int64_t ld64, float *__restrict__ D32, int64_t ld32,
                                        double *__restrict__ psi_out, double *dsh, int lane)
{
    const double *a = theta, *b = theta + V, *W = theta + V + H;
    const int64_t P1 = (int64_t)V * H + H + V + 1;
    const int baseW = V + H + 1;
    const float invV = 1.0f / (float)V;
    // x as a bit mask over v: alpha orbitals at v < n, beta at v = n + p
    uint64_t xm = (key & 0xffffffffull) | ((key >> 32) << n);
    double tsum = 0.0;
    for (int h = lane; h < H; h += kWave) {
        double z = b[h];
        for (uint64_t m = xm; m; m &= m - 1) z += W[(size_t)h * V + (__ffsll((unsigned long long)m) - 1)];
        double t = tanh(z);
        tsum += t;
        dsh[h] = 1.0 - t * t;
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
    const int64_t ldw = D64 ? ld64 : ld32;
    for (int64_t c0 = 2 * lane; c0 < ldw; c0 += 2 * kWave) {
        double val[2];
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            int64_t c = c0 + q;
            double x;
            if (c == 0) {
                x = psi;
            } else if (c <= V) {
                x = (double)((xm >> (c - 1)) & 1ull);
            } else if (c < baseW) {
                x = dsh[c - V - 1];
            } else if (c < P1) {
                int idx = (int)(c - baseW);
                int hh = (int)((float)idx * invV);
                int vv = idx - hh * V;
                if (vv < 0) { --hh; vv += V; }
                if (vv >= V) { ++hh; vv -= V; }
                x = ((xm >> vv) & 1ull) ? dsh[hh] : 0.0;
            } else {
                x = 0.0;
            }
            val[q] = x;
        }
        if (D64) {
            typedef double d2 __attribute__((ext_vector_type(2)));
            d2 v2 = {val[0], val[1]};
            __builtin_nontemporal_store(v2, (d2 *)(D64 + row * ld64 + c0));
        }
        if (D32 && c0 < ld32) {
            typedef float f2 __attribute__((ext_vector_type(2)));
            f2 v2 = {(float)val[0], (float)val[1]};
            __builtin_nontemporal_store(v2, (f2 *)(D32 + row * ld32 + c0));
        }
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__global__ __launch_bounds__(256) void k_nqs_dtilde(const uint64_t *__restrict__ keys, int64_t ns,
                                                    int n, int V, int H,
                                                    const double *__restrict__ theta,
                                                    double *__restrict__ D64, int64_t ld64,
                                                    float *__restrict__ D32, int64_t ld32,
                                                    double *__restrict__ psi_out)
{
    __shared__ double dsh[4][kMaxHidden];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t nwaves = (int64_t)gridDim.x * 4;
    for (int64_t row = (int64_t)blockIdx.x * 4 + wv; row < ns; row += nwaves)
        nqs_row(keys[row], row, n, V, H, theta, D64, ld64, D32, ld32, psi_out, dsh[wv], lane);
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
                mb.ld, const_cast<float *>(mb.D32), mb.ld, mb.psi, dsh[wv], lane);
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
    int64_t blocks = (L.ns + 3) / 4;
    if (blocks > 16384) blocks = 16384;
    k_nqs_dtilde<<<(unsigned)blocks, 256, 0, st>>>(s->d.keys, L.ns, s->n, V, H, theta, D64,
                                                   L.ld64, D32, L.ld32,
                                                   ws_ptr<double>(ws, L.off_psi));
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
