// Streams over D~ (HBM-bound) and the energy reductions, gfx950.
//
// The LM operator apply (Methods, "Practical Matrix-Free Implementation": the
// eigen-solver only needs matrix-vector products) reads D~ twice per vector:
//   K6  w = D~ v               one wavefront per row, v staged in LDS;
//   K7  [ya, yb] = D~^T [a, b] column tiles x row blocks, two right-hand sides
//                               per pass, per-block partial sums;
// followed by a two-level fixed-order reduction of the partials (no float
// atomics: results are bitwise reproducible).  D~ rows are read with 16-byte
// non-temporal loads, 1 KiB per wavefront instruction.  FP32 copies are
// multiplied and accumulated in FP32 inside a row block (the operator's
// reduced-precision mode); block partials are combined in FP64.
#include <algorithm>

#include "internal.h"

namespace irl {

typedef double d2 __attribute__((ext_vector_type(2)));
typedef float f4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------- K6: w = D v
template <typename T>
struct Chunk;
template <>
struct Chunk<double> {
    typedef d2 V;
    static constexpr int E = 2;
};
template <>
struct Chunk<float> {
    typedef f4 V;
    static constexpr int E = 4;
};

template <typename T>
__device__ __forceinline__ T dot_chunk(typename Chunk<T>::V x, const T *v)
{
    if constexpr (Chunk<T>::E == 2) {
        return x.x * v[0] + x.y * v[1];
    } else {
        return x.x * v[0] + x.y * v[1] + x.z * v[2] + x.w * v[3];
    }
}

constexpr size_t kMaxLdsBytes = 64 * 1024;

// rows [r0, r1) of D (row stride ld), interleaved over the 4 waves of a block:
// w[r] = D[r, :] . v, one wavefront per row, 4 x 16-byte loads in flight per lane
template <typename T>
__device__ __forceinline__ void gemv_rows_range(const T *__restrict__ D, int64_t ld, int64_t r0,
                                                int64_t r1, const T *vs, double *__restrict__ w,
                                                int lane, int wv)
{
    typedef typename Chunk<T>::V CV;
    constexpr int E = Chunk<T>::E;
    const int64_t nch = ld / E;               // chunks per row (ld is a multiple of E)
    for (int64_t r = r0 + wv; r < r1; r += 4) {
        const CV *row = reinterpret_cast<const CV *>(D + r * ld);
        T acc = 0;
        int64_t k = lane;
        for (; k + 3 * kWave < nch; k += 4 * kWave) {
            CV x0 = __builtin_nontemporal_load(row + k);
            CV x1 = __builtin_nontemporal_load(row + k + kWave);
            CV x2 = __builtin_nontemporal_load(row + k + 2 * kWave);
            CV x3 = __builtin_nontemporal_load(row + k + 3 * kWave);
            acc += dot_chunk<T>(x0, vs + k * E);
            acc += dot_chunk<T>(x1, vs + (k + kWave) * E);
            acc += dot_chunk<T>(x2, vs + (k + 2 * kWave) * E);
            acc += dot_chunk<T>(x3, vs + (k + 3 * kWave) * E);
        }
        for (; k < nch; k += kWave) acc += dot_chunk<T>(__builtin_nontemporal_load(row + k), vs + k * E);
        for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, kWave);
        if (lane == 0) w[r] = (double)acc;
    }
}

// VLDS: v staged in LDS (row length up to 64 KiB), else read through the caches
template <typename T, bool VLDS>
__global__ __launch_bounds__(256) void k_gemv_rows(const T *__restrict__ D, int64_t ld, int64_t ns,
                                                   const double *__restrict__ v, int64_t nv,
                                                   const T *__restrict__ vglob, int c0,
                                                   double *__restrict__ w)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const T *vs = vglob;
    if constexpr (VLDS) {
        T *vl = reinterpret_cast<T *>(smem_raw);
        for (int64_t c = threadIdx.x; c < ld; c += blockDim.x)
            vl[c] = (c < nv && c >= c0) ? (T)v[c] : (T)0;
        __syncthreads();
        vs = vl;
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    // contiguous row range per block, rows interleaved over the 4 waves
    const int64_t per = (ns + gridDim.x - 1) / gridDim.x;
    const int64_t r0 = (int64_t)blockIdx.x * per, r1 = min(ns, r0 + per);
    gemv_rows_range<T>(D, ld, r0, r1, vs, w, lane, wv);
}

// vector v converted to the stream precision, zero padded to ld
template <typename T>
__global__ void k_vec_convert(const double *__restrict__ v, int64_t nv, int64_t ld, int c0, T *out)
{
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < ld;
         c += (int64_t)gridDim.x * blockDim.x)
        out[c] = (c < nv && c >= c0) ? (T)v[c] : (T)0;
}

template <typename T>
static hipError_t gemv_rows_typed(const T *D, int64_t ld, int64_t ns, const double *v, int64_t nv,
                                  int c0, T *vtmp, double *w, hipStream_t st)
{
    const int64_t nblk = ns < 4096 ? (ns + 3) / 4 : 2048;
    const size_t sh = (size_t)ld * sizeof(T);
    if (sh <= kMaxLdsBytes) {
        k_gemv_rows<T, true><<<(unsigned)nblk, 256, sh, st>>>(D, ld, ns, v, nv, nullptr, c0, w);
    } else {
        k_vec_convert<T><<<(unsigned)((ld + 255) / 256), 256, 0, st>>>(v, nv, ld, c0, vtmp);
        k_gemv_rows<T, false><<<(unsigned)nblk, 256, 0, st>>>(D, ld, ns, v, nv, vtmp, c0, w);
    }
    return hipGetLastError();
}

hipError_t launch_gemv_rows(const WsLayout &L, void *ws, int prec, const double *v, double *w,
                            int zero_v0, hipStream_t st)
{
    // vconv holds the vector converted to the stream precision when it is too long for LDS
    const int c0 = zero_v0 ? 1 : 0;
    if (prec == IRL_FP64)
        return gemv_rows_typed<double>(ws_ptr<double>(ws, L.off_d64), L.ld64, L.ns, v, L.ncols, c0,
                                       ws_ptr<double>(ws, L.off_vconv), w, st);
    return gemv_rows_typed<float>(ws_ptr<float>(ws, L.off_d32), L.ld32, L.ns, v, L.ncols, c0,
                                  ws_ptr<float>(ws, L.off_vconv), w, st);
}

// ------------------------------------------------------ K7: [ya, yb] = D^T [a, b]
// b_r = b[r] - coef * sub[r] when sub != nullptr (coef read from device memory).
// Grid (column tiles, row blocks).  Each wavefront takes whole rows of its
// tile (lane owns chunks cbase + 64 q, q < NCH: every row issues NCH
// independent 16-byte loads per lane), the 4 wavefronts of a block are summed
// in LDS in a fixed order and the block writes one partial row.
// Rows [r0, r1) of column tile `tile` (lane owns chunks tile*64*NCH + lane +
// 64 q): acc_a += a_r D[r, :], acc_b += b_r D[r, :], b_r = b[r] - coef sub[r].
// Each column is summed by one lane over the wave's rows (r0 + wv + 4 t) and the
// 4 waves are combined ((w0 + w1) + w2) + w3, so the order per column does not
// depend on NCH.  Wave 0 writes the block's partial row (pa, pb).
template <typename T, int NCH>
__device__ __forceinline__ void gemv_t2_range(const T *__restrict__ D, int64_t ld, int64_t r0,
                                              int64_t r1, int tile, const double *__restrict__ a,
                                              const double *__restrict__ b,
                                              const double *__restrict__ sub, double coef,
                                              double *__restrict__ pa, double *__restrict__ pb,
                                              typename Chunk<T>::V (*red)[64 * NCH])
{
    typedef typename Chunk<T>::V CV;
    constexpr int E = Chunk<T>::E;
    const int64_t nch = ld / E;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t cbase = (int64_t)tile * 64 * NCH + lane;
    CV acc_a[NCH], acc_b[NCH];
#pragma unroll
    for (int q = 0; q < NCH; ++q) {
        acc_a[q] = (CV)0;
        acc_b[q] = (CV)0;
    }
    for (int64_t r = r0 + wv; r < r1; r += 4) {
        const double ad = a[r];
        const double bd = sub ? b[r] - coef * sub[r] : b[r];
        const T av = (T)ad, bv = (T)bd;
        const CV *row = reinterpret_cast<const CV *>(D + r * ld);
        CV x[NCH];
#pragma unroll
        for (int q = 0; q < NCH; ++q) {
            const int64_t k = cbase + (int64_t)q * 64;
            x[q] = k < nch ? __builtin_nontemporal_load(row + k) : (CV)0;
        }
#pragma unroll
        for (int q = 0; q < NCH; ++q) {
            acc_a[q] += av * x[q];
            acc_b[q] += bv * x[q];
        }
    }
    for (int src = 1; src < 4; ++src) {
        __syncthreads();
        if (wv == src) {
#pragma unroll
            for (int q = 0; q < NCH; ++q) {
                red[0][q * 64 + lane] = acc_a[q];
                red[1][q * 64 + lane] = acc_b[q];
            }
        }
        __syncthreads();
        if (wv == 0) {
#pragma unroll
            for (int q = 0; q < NCH; ++q) {
                acc_a[q] += red[0][q * 64 + lane];
                acc_b[q] += red[1][q * 64 + lane];
            }
        }
    }
    if (wv != 0) return;
#pragma unroll
    for (int q = 0; q < NCH; ++q) {
        const int64_t k = cbase + (int64_t)q * 64;
        if (k < nch) {
#pragma unroll
            for (int e = 0; e < E; ++e) {
                pa[k * E + e] = (double)acc_a[q][e];
                pb[k * E + e] = (double)acc_b[q][e];
            }
        }
    }
}

// K7 launch: grid (column tiles, row blocks); rows per block = ceil(ns / nblk)
template <typename T, int NCH>
__global__ __launch_bounds__(256) void k_gemv_t2(const T *__restrict__ D, int64_t ld, int64_t ns,
                                                 const double *__restrict__ a,
                                                 const double *__restrict__ b,
                                                 const double *__restrict__ sub,
                                                 const double *__restrict__ coefp,
                                                 double *__restrict__ part, int64_t ldv,
                                                 int nblk_rows, int rb0)
{
    typedef typename Chunk<T>::V CV;
    __shared__ CV red[2][64 * NCH];
    const int tile = blockIdx.x, rb = blockIdx.y + rb0;
    const int64_t per = (ns + nblk_rows - 1) / nblk_rows;
    const int64_t r0 = (int64_t)rb * per, r1 = min(ns, r0 + per);
    const double coef = sub ? *coefp : 0.0;
    double *pa = part + (int64_t)rb * 2 * ldv;
    gemv_t2_range<T, NCH>(D, ld, r0, r1, tile, a, b, sub, coef, pa, pa + ldv, red);
}

// stage 1: group g sums row blocks [g*per, (g+1)*per) of part -> part2[g]
__global__ void k_reduce_stage1(const double *__restrict__ part, int nblk, int64_t len,
                                double *__restrict__ part2, int groups)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int g = blockIdx.y;
    if (c >= len) return;
    const int per = (nblk + groups - 1) / groups;
    const int b0 = g * per, b1 = min(nblk, b0 + per);
    double s = 0.0;
    // unrolled so that the loads of 8 partial rows are in flight together (same order)
#pragma unroll 8
    for (int b = b0; b < b1; ++b) s += part[(int64_t)b * len + c];
    part2[(int64_t)g * len + c] = s;
}

// stage 2: out = scale / (div ? *div : 1) * sum_g part2[g]; first half -> ya, second -> yb
__global__ void k_reduce_stage2(const double *__restrict__ part2, int groups, int64_t ldv,
                                double *ya, double *yb, int64_t nout, double scale,
                                const double *divp)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= 2 * ldv) return;
    const int64_t cc = c < ldv ? c : c - ldv;
    if (cc >= nout) return;
    double s = 0.0;
    for (int g = 0; g < groups; ++g) s += part2[(int64_t)g * 2 * ldv + c];
    const double f = divp ? scale / *divp : scale;
    if (c < ldv) {
        if (ya) ya[cc] = s * f;
    } else {
        if (yb) yb[cc] = s * f;
    }
}

template <typename T, int NCH>
static void launch_t2_inst(const T *D, int64_t ld, int64_t ns, const double *a, const double *b,
                           const double *sub, const double *coef, double *part, int64_t ldv,
                           int ntiles, int nblk, int rbA, int rbB, hipStream_t st)
{
    k_gemv_t2<T, NCH><<<dim3(ntiles, rbB - rbA), 256, 0, st>>>(D, ld, ns, a, b, sub, coef, part, ldv,
                                                               nblk, rbA);
}

// row blocks of the D~^T launch for a row length ld (elements) and ns rows
template <typename T>
static int t2_row_blocks(int64_t ld, int64_t ns, int &ntiles, int &nch_lane)
{
    constexpr int E = Chunk<T>::E;
    const int64_t nch = ld / E;
    ntiles = (int)((nch + 64 * 16 - 1) / (64 * 16));
    nch_lane = (int)((nch + 64 * ntiles - 1) / (64 * ntiles));   // <= 16
    int nblk = kStreamBlocks / ntiles;
    if (nblk < 1) nblk = 1;
    if (nblk > (ns + 3) / 4) nblk = (int)((ns + 3) / 4);
    return nblk;
}

// row blocks [rbA, rbB) of the launch (rbB < 0: all); the partition into row
// blocks, and hence every partial sum, does not depend on the range launched
template <typename T>
static hipError_t launch_t2_typed(const T *D, int64_t ld, int64_t ns, const double *a,
                                  const double *b, const double *sub, const double *coef,
                                  double *part, int64_t ldv, int &nblk_out, int rbA, int rbB,
                                  hipStream_t st)
{
    int ntiles = 1, NCH = 16;
    const int nblk = t2_row_blocks<T>(ld, ns, ntiles, NCH);
    nblk_out = nblk;
    if (rbB < 0) rbB = nblk;
    if (rbA < 0 || rbB > nblk || rbA > rbB) return hipErrorInvalidValue;
    if (rbA == rbB) return hipSuccess;
#define T2CASE(c) case c: launch_t2_inst<T, c>(D, ld, ns, a, b, sub, coef, part, ldv, ntiles, nblk, rbA, rbB, st); break;
    switch (NCH) {
        T2CASE(1) T2CASE(2) T2CASE(3) T2CASE(4) T2CASE(5) T2CASE(6) T2CASE(7) T2CASE(8)
        T2CASE(9) T2CASE(10) T2CASE(11) T2CASE(12) T2CASE(13) T2CASE(14) T2CASE(15)
        default: launch_t2_inst<T, 16>(D, ld, ns, a, b, sub, coef, part, ldv, ntiles, nblk, rbA, rbB, st); break;
    }
#undef T2CASE
    return hipGetLastError();
}

int gemv_t2_row_blocks(const WsLayout &L, int prec)
{
    int ntiles, nch;
    return prec == IRL_FP64 ? t2_row_blocks<double>(L.ld64, L.ns, ntiles, nch)
                            : t2_row_blocks<float>(L.ld32, L.ns, ntiles, nch);
}

hipError_t launch_gemv_t2_blocks(const WsLayout &L, void *ws, int prec, const double *a,
                                 const double *b, const double *b_sub, const double *b_coef,
                                 int *nblk, int rbA, int rbB, hipStream_t st)
{
    double *part = ws_ptr<double>(ws, L.off_part);
    if (prec == IRL_FP64)
        return launch_t2_typed<double>(ws_ptr<double>(ws, L.off_d64), L.ld64, L.ns, a, b, b_sub,
                                       b_coef, part, L.ldv, *nblk, rbA, rbB, st);
    return launch_t2_typed<float>(ws_ptr<float>(ws, L.off_d32), L.ld32, L.ns, a, b, b_sub, b_coef,
                                  part, L.ldv, *nblk, rbA, rbB, st);
}

hipError_t launch_gemv_t2(const WsLayout &L, void *ws, int prec, const double *a,
                          const double *b, const double *b_sub, const double *b_coef,
                          int *nblk, hipStream_t st)
{
    return launch_gemv_t2_blocks(L, ws, prec, a, b, b_sub, b_coef, nblk, 0, -1, st);
}

hipError_t launch_t2_reduce(const WsLayout &L, void *ws, int nblk, double *ya, double *yb,
                            int64_t nout, double out_scale, const double *out_div, hipStream_t st)
{
    double *part = ws_ptr<double>(ws, L.off_part);
    double *part2 = ws_ptr<double>(ws, L.off_part2);
    const int64_t len = 2 * L.ldv;
    const int groups = nblk < kReduceGroups ? nblk : kReduceGroups;
    k_reduce_stage1<<<dim3((unsigned)((len + 255) / 256), groups), 256, 0, st>>>(part, nblk, len,
                                                                                 part2, groups);
    k_reduce_stage2<<<(unsigned)((len + 255) / 256), 256, 0, st>>>(part2, groups, L.ldv, ya, yb,
                                                                   nout, out_scale, out_div);
    return hipGetLastError();
}

// ------------------------------------------- multi-vector streams (nb <= 8)
// One pass over D~ serves nb vectors (the block operator of a block Lanczos
// step): K6 computes nb dot products per row from one set of 16-byte loads, K7
// carries 2 nb right-hand sides.  Bytes per pass stay those of one vector;
// arithmetic grows nb times and stays far below the HBM ridge for nb <= 8.

// W[q * ns + r] = D[r, :] . v_q (v_q staged in LDS, or converted vectors in global memory)
template <typename T, int NB, bool VLDS>
__global__ __launch_bounds__(256) void k_gemv_rows_multi(const T *__restrict__ D, int64_t ld, int64_t ns,
                                                         const double *__restrict__ V, int64_t ldv_in,
                                                         int64_t nv, const T *__restrict__ vglob, int c0,
                                                         double *__restrict__ W)
{
    typedef typename Chunk<T>::V CV;
    constexpr int E = Chunk<T>::E;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const T *vs = vglob;
    if constexpr (VLDS) {
        T *vl = reinterpret_cast<T *>(smem_raw);
        for (int64_t i = threadIdx.x; i < NB * ld; i += blockDim.x) {
            const int q = (int)(i / ld);
            const int64_t c = i - (int64_t)q * ld;
            vl[i] = (c < nv && c >= c0) ? (T)V[q * ldv_in + c] : (T)0;
        }
        __syncthreads();
        vs = vl;
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t nch = ld / E;
    const int64_t per = (ns + gridDim.x - 1) / gridDim.x;
    const int64_t r0 = (int64_t)blockIdx.x * per, r1 = min(ns, r0 + per);
    for (int64_t r = r0 + wv; r < r1; r += 4) {
        const CV *row = reinterpret_cast<const CV *>(D + r * ld);
        T acc[NB];
#pragma unroll
        for (int q = 0; q < NB; ++q) acc[q] = 0;
        int64_t k = lane;
        for (; k + kWave < nch; k += 2 * kWave) {
            const CV x0 = __builtin_nontemporal_load(row + k);
            const CV x1 = __builtin_nontemporal_load(row + k + kWave);
#pragma unroll
            for (int q = 0; q < NB; ++q) {
                acc[q] += dot_chunk<T>(x0, vs + q * ld + k * E);
                acc[q] += dot_chunk<T>(x1, vs + q * ld + (k + kWave) * E);
            }
        }
        for (; k < nch; k += kWave) {
            const CV x0 = __builtin_nontemporal_load(row + k);
#pragma unroll
            for (int q = 0; q < NB; ++q) acc[q] += dot_chunk<T>(x0, vs + q * ld + k * E);
        }
#pragma unroll
        for (int q = 0; q < NB; ++q) {
            T a = acc[q];
            for (int off = 32; off > 0; off >>= 1) a += __shfl_xor(a, off, kWave);
            if (lane == 0) W[q * ns + r] = (double)a;
        }
    }
}

// nb vectors converted to the stream precision, zero padded to ld (stride ld)
template <typename T>
__global__ void k_vec_convert_multi(const double *__restrict__ V, int64_t ldv_in, int nb, int64_t nv,
                                    int64_t ld, int c0, T *out)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nb * ld;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int q = (int)(i / ld);
        const int64_t c = i - (int64_t)q * ld;
        out[i] = (c < nv && c >= c0) ? (T)V[q * ldv_in + c] : (T)0;
    }
}

template <typename T, int NB>
static void gemv_rows_multi_inst(const T *D, int64_t ld, int64_t ns, const double *V, int64_t ldv_in,
                                 int64_t nv, int c0, T *vtmp, double *W, hipStream_t st)
{
    const int64_t nblk = ns < 4096 ? (ns + 3) / 4 : 2048;
    const size_t sh = (size_t)NB * ld * sizeof(T);
    if (sh <= kMaxLdsBytes) {
        k_gemv_rows_multi<T, NB, true><<<(unsigned)nblk, 256, sh, st>>>(D, ld, ns, V, ldv_in, nv, nullptr,
                                                                         c0, W);
    } else {
        k_vec_convert_multi<T><<<(unsigned)((NB * ld + 255) / 256), 256, 0, st>>>(V, ldv_in, NB, nv, ld, c0,
                                                                                  vtmp);
        k_gemv_rows_multi<T, NB, false><<<(unsigned)nblk, 256, 0, st>>>(D, ld, ns, V, ldv_in, nv, vtmp,
                                                                        c0, W);
    }
}

template <typename T>
static hipError_t gemv_rows_multi_typed(const T *D, int64_t ld, int64_t ns, const double *V,
                                        int64_t ldv_in, int nb, int64_t nv, int c0, T *vtmp, double *W,
                                        hipStream_t st)
{
    switch (nb) {
    case 1: gemv_rows_multi_inst<T, 1>(D, ld, ns, V, ldv_in, nv, c0, vtmp, W, st); break;
    case 2: gemv_rows_multi_inst<T, 2>(D, ld, ns, V, ldv_in, nv, c0, vtmp, W, st); break;
    case 3: gemv_rows_multi_inst<T, 3>(D, ld, ns, V, ldv_in, nv, c0, vtmp, W, st); break;
    case 4: gemv_rows_multi_inst<T, 4>(D, ld, ns, V, ldv_in, nv, c0, vtmp, W, st); break;
    case 5: gemv_rows_multi_inst<T, 5>(D, ld, ns, V, ldv_in, nv, c0, vtmp, W, st); break;
    case 6: gemv_rows_multi_inst<T, 6>(D, ld, ns, V, ldv_in, nv, c0, vtmp, W, st); break;
    case 7: gemv_rows_multi_inst<T, 7>(D, ld, ns, V, ldv_in, nv, c0, vtmp, W, st); break;
    case 8: gemv_rows_multi_inst<T, 8>(D, ld, ns, V, ldv_in, nv, c0, vtmp, W, st); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_gemv_rows_multi(const WsLayout &L, void *ws, int prec, const double *V, int64_t ldv_in,
                                  int nb, int zero_v0, double *W, hipStream_t st)
{
    if (nb < 1 || nb > layout_vectors(L)) return hipErrorInvalidValue;
    const int c0 = zero_v0 ? 1 : 0;
    if (prec == IRL_FP64)
        return gemv_rows_multi_typed<double>(ws_ptr<double>(ws, L.off_d64), L.ld64, L.ns, V, ldv_in, nb,
                                             L.ncols, c0, ws_ptr<double>(ws, L.off_vconv), W, st);
    return gemv_rows_multi_typed<float>(ws_ptr<float>(ws, L.off_d32), L.ld32, L.ns, V, ldv_in, nb, L.ncols,
                                        c0, ws_ptr<float>(ws, L.off_vconv), W, st);
}

// K7 with 2 NB right-hand sides: acc[2q] += W[q][r] D[r, :], acc[2q+1] += U[q][r] D[r, :].
// Rows [r0, r1) per block, NCH chunks per lane per column tile, the 4 waves combined
// ((w0 + w1) + w2) + w3; the block writes 2 NB partial rows: part[(rb*2NB + j) * ldv].
template <typename T, int NCH, int NB>
__global__ __launch_bounds__(256) void k_gemv_t2_multi(const T *__restrict__ D, int64_t ld, int64_t ns,
                                                       const double *__restrict__ W,
                                                       const double *__restrict__ U,
                                                       double *__restrict__ part, int64_t ldv, int nblk)
{
    typedef typename Chunk<T>::V CV;
    constexpr int E = Chunk<T>::E;
    __shared__ CV red[2 * NB][64 * NCH];
    const int tile = blockIdx.x, rb = blockIdx.y;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t nch = ld / E;
    const int64_t per = (ns + nblk - 1) / nblk;
    const int64_t r0 = (int64_t)rb * per, r1 = min(ns, r0 + per);
    const int64_t cbase = (int64_t)tile * 64 * NCH + lane;
    CV acc[2 * NB][NCH];
#pragma unroll
    for (int j = 0; j < 2 * NB; ++j)
#pragma unroll
        for (int c = 0; c < NCH; ++c) acc[j][c] = (CV)0;
    for (int64_t r = r0 + wv; r < r1; r += 4) {
        const CV *row = reinterpret_cast<const CV *>(D + r * ld);
        CV x[NCH];
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
            const int64_t k = cbase + (int64_t)c * 64;
            x[c] = k < nch ? __builtin_nontemporal_load(row + k) : (CV)0;
        }
#pragma unroll
        for (int q = 0; q < NB; ++q) {
            const T aq = (T)W[q * ns + r], bq = (T)U[q * ns + r];
#pragma unroll
            for (int c = 0; c < NCH; ++c) {
                acc[2 * q][c] += aq * x[c];
                acc[2 * q + 1][c] += bq * x[c];
            }
        }
    }
    for (int src = 1; src < 4; ++src) {
        __syncthreads();
        if (wv == src) {
#pragma unroll
            for (int j = 0; j < 2 * NB; ++j)
#pragma unroll
                for (int c = 0; c < NCH; ++c) red[j][c * 64 + lane] = acc[j][c];
        }
        __syncthreads();
        if (wv == 0) {
#pragma unroll
            for (int j = 0; j < 2 * NB; ++j)
#pragma unroll
                for (int c = 0; c < NCH; ++c) acc[j][c] += red[j][c * 64 + lane];
        }
    }
    if (wv != 0) return;
    double *prow = part + (int64_t)rb * 2 * NB * ldv;
#pragma unroll
    for (int j = 0; j < 2 * NB; ++j)
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
            const int64_t k = cbase + (int64_t)c * 64;
            if (k < nch) {
#pragma unroll
                for (int e = 0; e < E; ++e) prow[j * ldv + k * E + e] = (double)acc[j][c][e];
            }
        }
}

// chunks per lane per column tile for NB vectors (accumulators ~ 2 NB NCH chunks)
template <int NB>
constexpr int multi_nch() { return NB == 1 ? 16 : (NB == 2 ? 8 : (NB <= 4 ? 4 : 2)); }

// row blocks of the multi launch: about kStreamBlocks blocks in all, and at most
// kStreamBlocks * 2 partial rows (the size of the partial buffer)
static int multi_blocks(int64_t ns, int ntiles, int nb)
{
    int nblk = kStreamBlocks / ntiles;
    nblk = std::min(nblk, kStreamBlocks / nb);
    if (nblk < 1) nblk = 1;
    if (nblk > (ns + 3) / 4) nblk = (int)((ns + 3) / 4);
    return nblk;
}

template <typename T, int NB>
static void gemv_t2_multi_inst(const T *D, int64_t ld, int64_t ns, const double *W, const double *U,
                               double *part, int64_t ldv, int &nblk_out, hipStream_t st)
{
    constexpr int E = Chunk<T>::E;
    constexpr int NCH = multi_nch<NB>();
    const int64_t nch = ld / E;
    const int ntiles = (int)((nch + 64 * NCH - 1) / (64 * NCH));
    const int nblk = multi_blocks(ns, ntiles, NB);
    nblk_out = nblk;
    k_gemv_t2_multi<T, NCH, NB><<<dim3(ntiles, nblk), 256, 0, st>>>(D, ld, ns, W, U, part, ldv, nblk);
}

template <typename T>
static hipError_t gemv_t2_multi_typed(const T *D, int64_t ld, int64_t ns, int nb, const double *W,
                                      const double *U, double *part, int64_t ldv, int &nblk, hipStream_t st)
{
    switch (nb) {
    case 1: gemv_t2_multi_inst<T, 1>(D, ld, ns, W, U, part, ldv, nblk, st); break;
    case 2: gemv_t2_multi_inst<T, 2>(D, ld, ns, W, U, part, ldv, nblk, st); break;
    case 3: gemv_t2_multi_inst<T, 3>(D, ld, ns, W, U, part, ldv, nblk, st); break;
    case 4: gemv_t2_multi_inst<T, 4>(D, ld, ns, W, U, part, ldv, nblk, st); break;
    case 5: gemv_t2_multi_inst<T, 5>(D, ld, ns, W, U, part, ldv, nblk, st); break;
    case 6: gemv_t2_multi_inst<T, 6>(D, ld, ns, W, U, part, ldv, nblk, st); break;
    case 7: gemv_t2_multi_inst<T, 7>(D, ld, ns, W, U, part, ldv, nblk, st); break;
    case 8: gemv_t2_multi_inst<T, 8>(D, ld, ns, W, U, part, ldv, nblk, st); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_gemv_t2_multi(const WsLayout &L, void *ws, int prec, int nb, const double *W,
                                const double *U, int *nblk, hipStream_t st)
{
    if (nb < 1 || nb > layout_vectors(L)) return hipErrorInvalidValue;
    double *part = ws_ptr<double>(ws, L.off_part);
    if (prec == IRL_FP64)
        return gemv_t2_multi_typed<double>(ws_ptr<double>(ws, L.off_d64), L.ld64, L.ns, nb, W, U, part,
                                           L.ldv, *nblk, st);
    return gemv_t2_multi_typed<float>(ws_ptr<float>(ws, L.off_d32), L.ld32, L.ns, nb, W, U, part, L.ldv,
                                      *nblk, st);
}

// stage 2 of the multi reduction: partial row j = 2q (a-sums, -> YS[:, q]) or
// 2q + 1 (b-sums, -> YH[:, q]); columns >= nout are not written
__global__ void k_reduce_stage2_multi(const double *__restrict__ part2, int groups, int64_t ldv, int nb,
                                      double *YS, double *YH, int64_t ldy, int64_t nout)
{
    const int64_t len = 2 * (int64_t)nb * ldv;
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= len) return;
    const int j = (int)(c / ldv);
    const int64_t i = c - (int64_t)j * ldv;
    if (i >= nout) return;
    double s = 0.0;
    for (int g = 0; g < groups; ++g) s += part2[(int64_t)g * len + c];
    if (j & 1)
        YH[(int64_t)(j >> 1) * ldy + i] = s;
    else
        YS[(int64_t)(j >> 1) * ldy + i] = s;
}

hipError_t launch_t2_reduce_multi(const WsLayout &L, void *ws, int nblk, int nb, double *YS, double *YH,
                                  int64_t ldy, hipStream_t st)
{
    if (nb < 1 || nb > layout_vectors(L)) return hipErrorInvalidValue;
    double *part = ws_ptr<double>(ws, L.off_part);
    double *part2 = ws_ptr<double>(ws, L.off_part2);
    const int64_t len = 2 * (int64_t)nb * L.ldv;
    const int groups = nblk < kReduceGroups ? nblk : kReduceGroups;
    k_reduce_stage1<<<dim3((unsigned)((len + 255) / 256), groups), 256, 0, st>>>(part, nblk, len, part2,
                                                                                 groups);
    k_reduce_stage2_multi<<<(unsigned)((len + 255) / 256), 256, 0, st>>>(part2, groups, L.ldv, nb, YS, YH,
                                                                         ldy, L.ncols);
    return hipGetLastError();
}

// ------------------------------------------- energy: Z = psi.psi, N = psi.(H psi)
struct Neu {
    double s, c;
};
__device__ __forceinline__ Neu neu_add(Neu a, double x)
{
    double t = a.s + x;
    double bp = t - a.s;
    double err = (a.s - (t - bp)) + (x - bp);
    return Neu{t, a.c + err};
}
__device__ __forceinline__ Neu neu_merge(Neu a, Neu b)
{
    Neu r = neu_add(a, b.s);
    r.c += b.c;
    return r;
}

// compensated sums of psi_r^2 and psi_r (H psi)_r over rows [r0, r1) -> red[0..3]
__device__ void energy_stage1_body(const double *__restrict__ psi, const double *__restrict__ hpsi,
                                   int64_t r0, int64_t r1, double *__restrict__ red)
{
    __shared__ double sh[4][256];
    Neu z{0, 0}, e{0, 0};
    for (int64_t r = r0 + threadIdx.x; r < r1; r += blockDim.x) {
        double p = psi[r];
        z = neu_add(z, p * p);
        e = neu_add(e, p * hpsi[r]);
    }
    sh[0][threadIdx.x] = z.s;
    sh[1][threadIdx.x] = z.c;
    sh[2][threadIdx.x] = e.s;
    sh[3][threadIdx.x] = e.c;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            Neu a{sh[0][threadIdx.x], sh[1][threadIdx.x]}, b{sh[0][threadIdx.x + w], sh[1][threadIdx.x + w]};
            Neu c{sh[2][threadIdx.x], sh[3][threadIdx.x]}, d{sh[2][threadIdx.x + w], sh[3][threadIdx.x + w]};
            a = neu_merge(a, b);
            c = neu_merge(c, d);
            sh[0][threadIdx.x] = a.s;
            sh[1][threadIdx.x] = a.c;
            sh[2][threadIdx.x] = c.s;
            sh[3][threadIdx.x] = c.c;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        red[0] = sh[0][0];
        red[1] = sh[1][0];
        red[2] = sh[2][0];
        red[3] = sh[3][0];
    }
}

__global__ __launch_bounds__(256) void k_energy_stage1(const double *__restrict__ psi,
                                                       const double *__restrict__ hpsi, int64_t ns,
                                                       double *__restrict__ red)
{
    const int64_t per = (ns + gridDim.x - 1) / gridDim.x;
    const int64_t r0 = (int64_t)blockIdx.x * per, r1 = min(ns, r0 + per);
    energy_stage1_body(psi, hpsi, r0, r1, red + blockIdx.x * 4);
}

// one wavefront (64 threads): lane l merges parts l, l + 64, ... in order, then a
// fixed halving tree (lane l takes lane l + off) leaves the total on lane 0
__device__ void energy_stage2_body(const double *__restrict__ red, int nparts, WsScalars *sc)
{
    const int lane = threadIdx.x;
    if (lane >= kWave) return;
    Neu z{0, 0}, e{0, 0};
    for (int i = lane; i < nparts; i += kWave) {
        z = neu_merge(z, Neu{red[i * 4 + 0], red[i * 4 + 1]});
        e = neu_merge(e, Neu{red[i * 4 + 2], red[i * 4 + 3]});
    }
    for (int off = kWave / 2; off > 0; off >>= 1) {
        const Neu zo{__shfl_down(z.s, off, kWave), __shfl_down(z.c, off, kWave)};
        const Neu eo{__shfl_down(e.s, off, kWave), __shfl_down(e.c, off, kWave)};
        z = neu_merge(z, zo);
        e = neu_merge(e, eo);
    }
    if (lane != 0) return;
    sc->sum_psi2[0] = z.s;
    sc->sum_psi2[1] = z.c;
    sc->sum_psih[0] = e.s;
    sc->sum_psih[1] = e.c;
    const double Z = z.s + z.c, N = e.s + e.c;
    sc->Z = Z;
    sc->E_el = N / Z;
}

__global__ void k_energy_stage2(const double *__restrict__ red, int nparts, WsScalars *sc)
{
    energy_stage2_body(red, nparts, sc);
}

hipError_t launch_energy_reduce(const WsLayout &L, void *ws, hipStream_t st)
{
    int parts = L.ns < (int64_t)kScalarParts * 256 ? (int)((L.ns + 255) / 256) : kScalarParts;
    double *red = ws_ptr<double>(ws, L.off_red);
    k_energy_stage1<<<parts, 256, 0, st>>>(ws_ptr<double>(ws, L.off_psi),
                                           ws_ptr<double>(ws, L.off_hpsi), L.ns, red);
    k_energy_stage2<<<1, 64, 0, st>>>(red, parts, ws_ptr<WsScalars>(ws, L.off_scal));
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Grouped launches (batch): work item (member, indices, rows) per block, with
// the per-member arithmetic of the solo launches (same row blocks, same
// reduction order), so a batched result equals the solo result bit for bit.
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ const T *member_D(const Member &mb)
{
    if constexpr (sizeof(T) == 8)
        return reinterpret_cast<const T *>(mb.D64);
    else
        return reinterpret_cast<const T *>(mb.D32);
}

// vsel 0: v = Krylov row j of buffer cur; vsel 1: v = the Ritz vector y
template <typename T>
__global__ __launch_bounds__(256) void k_gemv_rows_grouped(const Member *__restrict__ M,
                                                           const WorkItem *__restrict__ items,
                                                           int vsel, int j, int cur, int c0)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const WorkItem it = items[blockIdx.x];
    const Member &mb = M[it.m];
    const double *v = vsel ? mb.y : mb.kry[cur] + (int64_t)j * mb.ld;
    T *vl = reinterpret_cast<T *>(smem_raw);
    for (int64_t c = threadIdx.x; c < mb.ld; c += blockDim.x)
        vl[c] = (c < mb.ncols && c >= c0) ? (T)v[c] : (T)0;
    __syncthreads();
    gemv_rows_range<T>(member_D<T>(mb), mb.ld, it.r0, it.r1, vl, mb.w, threadIdx.x & 63,
                       threadIdx.x >> 6);
}

hipError_t launch_gemv_rows_grouped(const Member *M, const WorkItem *items, int nitems, int prec,
                                    int vsel, int j, int cur, int zero_v0, size_t lds_bytes,
                                    hipStream_t st)
{
    if (nitems <= 0) return hipSuccess;
    if (prec == IRL_FP64)
        k_gemv_rows_grouped<double><<<nitems, 256, lds_bytes, st>>>(M, items, vsel, j, cur, zero_v0);
    else
        k_gemv_rows_grouped<float><<<nitems, 256, lds_bytes, st>>>(M, items, vsel, j, cur, zero_v0);
    return hipGetLastError();
}

// which 0: [yS, yH] partials of D~^T [w, u]; which 1: gradient partials of D~^T [psi, H psi - E psi]
template <typename T>
__global__ __launch_bounds__(256) void k_gemv_t2_grouped(const Member *__restrict__ M,
                                                         const WorkItem *__restrict__ items,
                                                         int which)
{
    typedef typename Chunk<T>::V CV;
    __shared__ CV red[2][64 * kGroupedT2Chunks];
    const WorkItem it = items[blockIdx.x];
    const Member &mb = M[it.m];
    const double *a = which ? mb.psi : mb.w;
    const double *b = which ? mb.hpsi : mb.u;
    const double *sub = which ? mb.psi : nullptr;
    const double coef = which ? mb.sc->E_el : 0.0;
    double *pa = mb.part + (int64_t)it.b * 2 * mb.ld;
    gemv_t2_range<T, kGroupedT2Chunks>(member_D<T>(mb), mb.ld, it.r0, it.r1, it.a, a, b, sub, coef,
                                       pa, pa + mb.ld, red);
}

hipError_t launch_gemv_t2_grouped(const Member *M, const WorkItem *items, int nitems, int prec,
                                  int which, hipStream_t st)
{
    if (nitems <= 0) return hipSuccess;
    if (prec == IRL_FP64)
        k_gemv_t2_grouped<double><<<nitems, 256, 0, st>>>(M, items, which);
    else
        k_gemv_t2_grouped<float><<<nitems, 256, 0, st>>>(M, items, which);
    return hipGetLastError();
}

// item: member m, column chunk a (256 of the 2 ld partial columns); the two
// reduction levels of the solo launch, in the same order
__global__ void k_reduce_grouped(const Member *__restrict__ M, const WorkItem *__restrict__ items,
                                 int which)
{
    const WorkItem it = items[blockIdx.x];
    const Member &mb = M[it.m];
    const int64_t len = 2 * mb.ld;
    const int64_t c = (int64_t)it.a * blockDim.x + threadIdx.x;
    if (c >= len) return;
    const int64_t cc = c < mb.ld ? c : c - mb.ld;
    if (cc >= mb.ncols) return;
    const int nblk = mb.nblk_t2;
    const int groups = nblk < kReduceGroups ? nblk : kReduceGroups;
    const int per = (nblk + groups - 1) / groups;
    double tot = 0.0;
    for (int g = 0; g < groups; ++g) {
        const int b0 = g * per, b1 = min(nblk, b0 + per);
        double s = 0.0;
#pragma unroll 8
        for (int b = b0; b < b1; ++b) s += mb.part[(int64_t)b * len + c];
        tot += s;
    }
    if (which == 0) {
        if (c < mb.ld) mb.yS[cc] = tot * 1.0;
        else mb.yH[cc] = tot * 1.0;
    } else {
        const double f = 2.0 / mb.sc->Z;
        if (c < mb.ld) mb.y[cc] = tot * f;
        else mb.grad[cc] = tot * f;
    }
}

hipError_t launch_reduce_grouped(const Member *M, const WorkItem *items, int nitems, int which,
                                 hipStream_t st)
{
    if (nitems <= 0) return hipSuccess;
    k_reduce_grouped<<<nitems, 256, 0, st>>>(M, items, which);
    return hipGetLastError();
}

// stage 1 item: member m, part a, rows [r0, r1); stage 2 item: member m
__global__ __launch_bounds__(256) void k_energy_grouped1(const Member *__restrict__ M,
                                                         const WorkItem *__restrict__ items)
{
    const WorkItem it = items[blockIdx.x];
    const Member &mb = M[it.m];
    energy_stage1_body(mb.psi, mb.hpsi, it.r0, it.r1, mb.red + (int64_t)it.a * 4);
}

__global__ void k_energy_grouped2(const Member *__restrict__ M, const WorkItem *__restrict__ items)
{
    const Member &mb = M[items[blockIdx.x].m];
    energy_stage2_body(mb.red, mb.nparts_e, mb.sc);
}

hipError_t launch_energy_grouped(const Member *M, const WorkItem *items, int nitems, int stage,
                                 hipStream_t st)
{
    if (nitems <= 0) return hipSuccess;
    if (stage == 1)
        k_energy_grouped1<<<nitems, 256, 0, st>>>(M, items);
    else
        k_energy_grouped2<<<nitems, 64, 0, st>>>(M, items);
    return hipGetLastError();
}

}  // namespace irl
