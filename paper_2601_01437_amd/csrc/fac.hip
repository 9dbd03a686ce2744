// Factored Jacobian of the one-hidden-layer network on gfx950 FP64 matrix cores.
//
// The rows of D~ are [psi, x, d, d (x) x] with d_h = 1 - t_h^2 (Methods, "From SR
// to a Stable Eigenvalue Problem": the tangent vectors are psi and its parameter
// derivatives), so every product with D~ reduces to contractions with the 0/1
// occupation matrix X (N_s x V) and the stored d (N_s x H):
//   forward   z = X W^T + b,  t = tanh z,  d = 1 - t^2,  psi = X a + sum_h t
//   D~ v      w_r = psi_r v_0 + x_r . v_a + sum_h d_rh (v_b[h] + (X V_W^T)_rh)
//   D~^T c    [sum c psi, X^T c, d^T c, ((c d)^T X)_hv]
// X W^T and (c d)^T X run on v_mfma_f64_16x16x4f64 (the dense FP64 contraction of
// the method: N_s V H multiply-adds per product); the rest is elementwise.
//
// Operand layout of the 16x16x4 FP64 MFMA (lane l, one wavefront): the lane
// supplies A[l % 16][l / 16] and B[l / 16][l % 16] and receives D[4 r + l / 16][l % 16]
// in register r.  Hidden units are relabelled inside a 64-wide chunk t so that
// lane l owns the 4 consecutive units h = 64 t + 4 (l % 16) + q of its column or row
// index: its d loads and stores are 32 contiguous bytes (chunks of 16 QT units with
// QT units per lane where the operands of 64 units would not fit the registers).
#include "internal.h"

#include <utility>

namespace irl {

typedef double d4v __attribute__((ext_vector_type(4)));
typedef double d2v __attribute__((ext_vector_type(2)));

__device__ __forceinline__ d4v mfma_f64(double a, double b, d4v c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// occupation bits over v: alpha orbitals at v < n, beta at v = n + p
__device__ __forceinline__ uint64_t occ_bits(uint64_t key, int n)
{
    return (key & 0xffffffffull) | ((key >> 32) << n);
}

// d[row][h0 .. h0 + QT) (zero past H); VEC: H % QT == 0, so the 8 QT bytes are aligned
template <int QT, bool VEC>
__device__ __forceinline__ void load_dq(const double *__restrict__ dfac, int64_t row, int H, int h0, double (&d)[QT])
{
    const double *p = dfac + row * H + h0;
    if (QT >= 2 && VEC && h0 < H) {
#pragma unroll
        for (int q = 0; q + 1 < QT; q += 2) {
            const d2v t = *(const d2v *)(p + q);
            d[q] = t.x;
            d[q + 1] = t.y;
        }
    } else {
#pragma unroll
        for (int q = 0; q < QT; ++q) d[q] = h0 + q < H ? p[q] : 0.0;
    }
}

template <int QT, bool VEC>
__device__ __forceinline__ void store_dq(double *__restrict__ dfac, int64_t row, int H, int h0, const double (&d)[QT])
{
    double *p = dfac + row * H + h0;
    if (QT >= 2 && VEC && h0 < H) {
#pragma unroll
        for (int q = 0; q + 1 < QT; q += 2) *(d2v *)(p + q) = d2v{d[q], d[q + 1]};
    } else {
#pragma unroll
        for (int q = 0; q < QT; ++q)
            if (h0 + q < H) p[q] = d[q];
    }
}

// B operand of Z = X M^T for hidden chunk t of 16 QT units (M: H x V, row-major):
// for k-step kk and column tile q the lane holds M[h][v] at v = 4 kk + l / 16,
// h = 16 QT t + QT (l % 16) + q (zero outside v < V, h < H).
template <int KS, int QT>
__device__ __forceinline__ void load_bt(const double *__restrict__ M, int V, int H, int t, int lane,
                                        double (&B)[KS][QT])
{
    const int vs = lane >> 4, h0 = 16 * QT * t + QT * (lane & 15);
#pragma unroll
    for (int kk = 0; kk < KS; ++kk)
#pragma unroll
        for (int q = 0; q < QT; ++q) {
            const int v = 4 * kk + vs, h = h0 + q;
            B[kk][q] = (v < V && h < H) ? M[(size_t)h * V + v] : 0.0;
        }
}

// Z for the 16 rows of a tile (the lane's A row is l % 16, occupation bits xa)
// and the 16 QT hidden units of the chunk: acc[q][r] = Z[4 r + l / 16][16 QT t + QT (l % 16) + q]
template <int KS, int QT>
__device__ __forceinline__ void z_tile(uint64_t xa, int lane, const double (&B)[KS][QT], d4v (&acc)[QT])
{
    const int vs = lane >> 4;
#pragma unroll
    for (int q = 0; q < QT; ++q) acc[q] = d4v{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int kk = 0; kk < KS; ++kk) {
        const double a = (double)(uint32_t)((xa >> (4 * kk + vs)) & 1ull);
#pragma unroll
        for (int q = 0; q < QT; ++q) acc[q] = mfma_f64(a, B[kk][q], acc[q]);
    }
}

// t = tanh z and d = 1 - t^2 from one expm1 of 2|z|: with e = expm1(2 |z|) >= 0,
// |t| = e / (e + 2) and 1 - t^2 = 4 (e + 1) / (e + 2)^2, which has no cancellation as
// |t| -> 1; |z| is capped at 354, where e is still finite and d is below 2e-307
__device__ __forceinline__ void tanh_and_d(double z, double &t, double &d)
{
    const double e = expm1(2.0 * fmin(fabs(z), 354.0));
    const double r = 1.0 / (e + 2.0);
    t = copysign(e * r, z);
    d = 4.0 * ((e + 1.0) * r) * r;
}

// x_r . u for the lane's A row (l % 16): partial over the lane's k-steps, then the
// four lanes of the row are added (every lane of the row ends with the total)
template <int KS>
__device__ __forceinline__ double x_dot(uint64_t xa, int lane, const double (&uk)[KS])
{
    const int vs = lane >> 4;
    double s = 0.0;
#pragma unroll
    for (int kk = 0; kk < KS; ++kk) s += ((xa >> (4 * kk + vs)) & 1ull) ? uk[kk] : 0.0;
    s += __shfl_xor(s, 16, kWave);
    s += __shfl_xor(s, 32, kWave);
    return s;
}

// per-row sums p[r] (row 4 r + l / 16) over the 16 lanes of each quarter, handed to
// lane j < 16 as the sum of row j
__device__ __forceinline__ double rows_to_lanes(double (&p)[4], int lane)
{
#pragma unroll
    for (int r = 0; r < 4; ++r)
        for (int off = 1; off < 16; off <<= 1) p[r] += __shfl_xor(p[r], off, kWave);
    const int j = lane & 15, src = 16 * (j & 3);
    double out = 0.0;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const double v = __shfl(p[r], src, kWave);
        if ((j >> 2) == r) out = v;
    }
    return out;
}

// ---------------------------------------------------------------------------
// forward pass: psi (N_s) and d (N_s x H) from theta = [a, b, W]; hidden chunks of
// 16 QT units
template <int KS, int QT, bool VEC>
__global__ __launch_bounds__(256) void k_fac_forward(const uint64_t *__restrict__ keys, int64_t ns, int n,
                                                     int V, int H, const double *__restrict__ theta,
                                                     double *__restrict__ psi, double *__restrict__ dfac)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t ntile = (ns + 15) / 16, nw = (int64_t)gridDim.x * 4;
    const double *a = theta, *b = theta + V, *W = theta + V + H;
    double ak[KS];
#pragma unroll
    for (int kk = 0; kk < KS; ++kk) {
        const int v = 4 * kk + (lane >> 4);
        ak[kk] = v < V ? a[v] : 0.0;
    }
    const int htiles = (H + 16 * QT - 1) / (16 * QT);
    for (int t = 0; t < htiles; ++t) {
        double B[KS][QT], bh[QT];
        load_bt<KS, QT>(W, V, H, t, lane, B);
        const int h0 = 16 * QT * t + QT * (lane & 15);
#pragma unroll
        for (int q = 0; q < QT; ++q) bh[q] = h0 + q < H ? b[h0 + q] : 0.0;
        for (int64_t tile = (int64_t)blockIdx.x * 4 + wv; tile < ntile; tile += nw) {
            const int64_t r0 = tile * 16, ra = r0 + (lane & 15);
            const uint64_t xa = ra < ns ? occ_bits(keys[ra], n) : 0ull;
            d4v acc[QT];
            z_tile<KS, QT>(xa, lane, B, acc);
            double ts[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t row = r0 + 4 * r + (lane >> 4);
                double d[QT], sum = 0.0;
#pragma unroll
                for (int q = 0; q < QT; ++q) {
                    double th;
                    tanh_and_d(acc[q][r] + bh[q], th, d[q]);
                    sum += h0 + q < H ? th : 0.0;
                }
                if (row < ns) store_dq<QT, VEC>(dfac, row, H, h0, d);
                ts[r] = sum;
            }
            double pj = rows_to_lanes(ts, lane);
            if (t == 0) pj += x_dot<KS>(xa, lane, ak);
            if (lane < 16 && ra < ns) psi[ra] = (t == 0 ? 0.0 : psi[ra]) + pj;
        }
    }
}

// ---------------------------------------------------------------------------
// w = D~ v with v = [v_0, v_a, v_b, V_W] (v_0 taken as 0 when zero_v0); hidden
// chunks of 16 QT units, the d rows and key of the next tile loaded while the
// current one is multiplied
template <int KS, int QT, bool VEC>
__global__ __launch_bounds__(256) void k_fac_jvp(const uint64_t *__restrict__ keys, int64_t ns, int n, int V,
                                                 int H, const double *__restrict__ dfac,
                                                 const double *__restrict__ psi, const double *__restrict__ v,
                                                 int zero_v0, double *__restrict__ w)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t ntile = (ns + 15) / 16, nw = (int64_t)gridDim.x * 4;
    const double *va = v + 1, *vb = v + 1 + V, *vW = v + 1 + V + H;
    const double v0 = zero_v0 ? 0.0 : v[0];
    double ak[KS];
#pragma unroll
    for (int kk = 0; kk < KS; ++kk) {
        const int vv = 4 * kk + (lane >> 4);
        ak[kk] = vv < V ? va[vv] : 0.0;
    }
    const int htiles = (H + 16 * QT - 1) / (16 * QT);
    for (int t = 0; t < htiles; ++t) {
        double B[KS][QT], bh[QT];
        load_bt<KS, QT>(vW, V, H, t, lane, B);
        const int h0 = 16 * QT * t + QT * (lane & 15);
#pragma unroll
        for (int q = 0; q < QT; ++q) bh[q] = h0 + q < H ? vb[h0 + q] : 0.0;
        auto fetch = [&](int64_t tile, double (&d)[4][QT], uint64_t &xa) {
            const int64_t r0 = tile * 16, ra = r0 + (lane & 15);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t row = r0 + 4 * r + (lane >> 4);
                if (row < ns) {
                    load_dq<QT, VEC>(dfac, row, H, h0, d[r]);
                } else {
#pragma unroll
                    for (int q = 0; q < QT; ++q) d[r][q] = 0.0;
                }
            }
            xa = ra < ns ? occ_bits(keys[ra], n) : 0ull;
        };
        double d[4][QT], dn[4][QT];
        uint64_t xa = 0ull, xn = 0ull;
        int64_t tile = (int64_t)blockIdx.x * 4 + wv;
        if (tile < ntile) fetch(tile, d, xa);
        for (; tile < ntile; tile += nw) {
            const int64_t r0 = tile * 16, ra = r0 + (lane & 15);
            if (tile + nw < ntile) fetch(tile + nw, dn, xn);
            d4v acc[QT];
            z_tile<KS, QT>(xa, lane, B, acc);
            double p[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                double sum = 0.0;
#pragma unroll
                for (int q = 0; q < QT; ++q) sum += d[r][q] * (acc[q][r] + bh[q]);
                p[r] = sum;
            }
            double pj = rows_to_lanes(p, lane);
            if (t == 0) {
                pj += x_dot<KS>(xa, lane, ak);
                if (lane < 16 && ra < ns) pj += psi[ra] * v0;
            }
            if (lane < 16 && ra < ns) w[ra] = (t == 0 ? 0.0 : w[ra]) + pj;
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int q = 0; q < QT; ++q) d[r][q] = dn[r][q];
            xa = xn;
        }
    }
}

// ---------------------------------------------------------------------------
// partial rows of D~^T c for NR right-hand sides c_r = y_r - coef psi_r (coef = 0
// without coefp): NR = 1 writes half `half` of each row block's pair of partial
// rows, NR = 2 writes c = y0 into half 0 and c = y1 into half 1 from one pass over
// d.  Grid (hidden chunks of CW = 16 MT units, row blocks); each wave takes
// groups of 4 rows (the K of the matrix product), loading the next group while
// the current one is multiplied.  A[h][k] = c_k d_kh (MT column tiles of 16 hidden
// units, lane l owning units MT (l % 16) + m of the chunk), B[k][v] = x_kv;
// the b entries (sum c d), the a entries (sum c x) and the psi entry (sum c psi)
// are lane-local sums beside the product.  The 4 waves are combined in a fixed
// order and wave 0 writes the entries of the partial rows that belong to its
// chunk (chunk 0 also the psi, a and padding entries).
template <int NT, int NR, int MT, bool VEC>
__global__ __launch_bounds__(256) void k_fac_vjp(const uint64_t *__restrict__ keys, int64_t ns, int n, int V,
                                                 int H, const double *__restrict__ dfac,
                                                 const double *__restrict__ psi, const double *__restrict__ y0,
                                                 const double *__restrict__ y1, const double *__restrict__ coefp,
                                                 double *__restrict__ part, int64_t ldv, int nblk, int half)
{
    constexpr int CW = 16 * MT;
    static_assert(NR * MT * NT <= 8, "accumulator tiles per lane");
    constexpr int kAcc = 4 * NR * MT * NT + NR * (MT + NT + 1);   // doubles per lane in the wave combination
    __shared__ double red[64 * kAcc];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int ht = blockIdx.x, rb = blockIdx.y;
    const int64_t per = (ns + nblk - 1) / nblk;
    const int64_t r0 = (int64_t)rb * per, r1 = min(ns, r0 + per);
    const double coef = coefp ? *coefp : 0.0;
    const int kq = lane >> 4, i = lane & 15, h0 = CW * ht + MT * i;
    const double *ys[2] = {y0, y1};
    d4v acc[NR][MT][NT];
    double accB[NR][MT], accA[NR][NT], acc0[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        acc0[r] = 0.0;
#pragma unroll
        for (int m = 0; m < MT; ++m) {
            accB[r][m] = 0.0;
#pragma unroll
            for (int nn = 0; nn < NT; ++nn) acc[r][m][nn] = d4v{0.0, 0.0, 0.0, 0.0};
        }
#pragma unroll
        for (int nn = 0; nn < NT; ++nn) accA[r][nn] = 0.0;
    }
    // one 4-row group: the lane's row is g + kq
    struct Grp {
        double d[MT], ps, y[NR];
        uint64_t x;
    };
    auto fetch = [&](int64_t g, Grp &q) {
        const int64_t row = g + kq;
        q.ps = 0.0;
        q.x = 0ull;
#pragma unroll
        for (int r = 0; r < NR; ++r) q.y[r] = 0.0;
#pragma unroll
        for (int m = 0; m < MT; ++m) q.d[m] = 0.0;
        if (row < r1) {
            load_dq<MT, VEC>(dfac, row, H, h0, q.d);
            q.ps = psi[row];
#pragma unroll
            for (int r = 0; r < NR; ++r) q.y[r] = ys[r][row];
            q.x = occ_bits(keys[row], n);
        }
    };
    auto consume = [&](const Grp &cur) {
        double Bv[NT];
#pragma unroll
        for (int nn = 0; nn < NT; ++nn) Bv[nn] = (double)(uint32_t)((cur.x >> (16 * nn + i)) & 1ull);
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            const double c = cur.y[r] - coef * cur.ps;
#pragma unroll
            for (int m = 0; m < MT; ++m) {
                const double A = c * cur.d[m];
                accB[r][m] += A;
#pragma unroll
                for (int nn = 0; nn < NT; ++nn) acc[r][m][nn] = mfma_f64(A, Bv[nn], acc[r][m][nn]);
            }
            if (ht == 0) {
#pragma unroll
                for (int nn = 0; nn < NT; ++nn) accA[r][nn] += c * Bv[nn];
                acc0[r] += c * cur.ps;
            }
        }
    };
    // ring of PD groups in flight per wave: a group is consumed, then its slot is
    // refilled with the group PD steps ahead (rows past r1 load as zeros)
    constexpr int PD = NT == 2 ? 8 : 4;   // deepest ring that keeps 2 or more waves per SIMD
    Grp ring[PD];
    const int64_t g0 = r0 + 4 * wv;
#pragma unroll
    for (int p = 0; p < PD; ++p) fetch(g0 + 16 * p, ring[p]);
    for (int64_t g = g0; g < r1; g += 16 * PD) {
#pragma unroll
        for (int p = 0; p < PD; ++p) {
            if (g + 16 * p < r1) consume(ring[p]);
            fetch(g + 16 * (p + PD), ring[p]);
        }
    }
    // sums over the 4 rows of a group (the lane quarters)
#pragma unroll
    for (int r = 0; r < NR; ++r) {
#pragma unroll
        for (int m = 0; m < MT; ++m) {
            accB[r][m] += __shfl_xor(accB[r][m], 16, kWave);
            accB[r][m] += __shfl_xor(accB[r][m], 32, kWave);
        }
#pragma unroll
        for (int nn = 0; nn < NT; ++nn) {
            accA[r][nn] += __shfl_xor(accA[r][nn], 16, kWave);
            accA[r][nn] += __shfl_xor(accA[r][nn], 32, kWave);
        }
        acc0[r] += __shfl_xor(acc0[r], 16, kWave);
        acc0[r] += __shfl_xor(acc0[r], 32, kWave);
    }

    // fixed-order combination of the 4 waves: ((w0 + w1) + w2) + w3
    auto slot = [&](int k) -> double & { return red[64 * k + lane]; };
    for (int src = 1; src < 4; ++src) {
        __syncthreads();
        if (wv == src || wv == 0) {
            const bool put = wv == src;
            int k = 0;
#pragma unroll
            for (int r = 0; r < NR; ++r) {
#pragma unroll
                for (int m = 0; m < MT; ++m)
#pragma unroll
                    for (int nn = 0; nn < NT; ++nn)
#pragma unroll
                        for (int q = 0; q < 4; ++q, ++k) {
                            if (put) slot(k) = acc[r][m][nn][q];
                        }
            }
#pragma unroll
            for (int r = 0; r < NR; ++r) {
#pragma unroll
                for (int m = 0; m < MT; ++m, ++k)
                    if (put) slot(k) = accB[r][m];
#pragma unroll
                for (int nn = 0; nn < NT; ++nn, ++k)
                    if (put) slot(k) = accA[r][nn];
                if (put) slot(k) = acc0[r];
                ++k;
            }
        }
        __syncthreads();
        if (wv == 0) {
            int k = 0;
#pragma unroll
            for (int r = 0; r < NR; ++r)
#pragma unroll
                for (int m = 0; m < MT; ++m)
#pragma unroll
                    for (int nn = 0; nn < NT; ++nn)
#pragma unroll
                        for (int q = 0; q < 4; ++q, ++k) acc[r][m][nn][q] += slot(k);
#pragma unroll
            for (int r = 0; r < NR; ++r) {
#pragma unroll
                for (int m = 0; m < MT; ++m, ++k) accB[r][m] += slot(k);
#pragma unroll
                for (int nn = 0; nn < NT; ++nn, ++k) accA[r][nn] += slot(k);
                acc0[r] += slot(k);
                ++k;
            }
        }
    }
    if (wv != 0) return;
    const int64_t baseW = 1 + V + H, P1 = (int64_t)V * H + H + V + 1;
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        double *out = part + ((int64_t)rb * 2 + (NR == 2 ? r : half)) * ldv;
        // acc[r][m][nn][q] = sum c d_h x_v at h = CW ht + MT (4 q + l / 16) + m, v = 16 nn + l % 16
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int m = 0; m < MT; ++m) {
                const int h = CW * ht + MT * (4 * q + kq) + m;
                if (h < H)
#pragma unroll
                    for (int nn = 0; nn < NT; ++nn) {
                        const int vv = 16 * nn + i;
                        if (vv < V) out[baseW + (int64_t)h * V + vv] = acc[r][m][nn][q];
                    }
            }
        if (lane < 16) {
#pragma unroll
            for (int m = 0; m < MT; ++m)
                if (h0 + m < H) out[1 + V + h0 + m] = accB[r][m];
            if (ht == 0) {
#pragma unroll
                for (int nn = 0; nn < NT; ++nn)
                    if (16 * nn + lane < V) out[1 + 16 * nn + lane] = accA[r][nn];
            }
        }
        if (ht == 0) {
            if (lane == 0) out[0] = acc0[r];
            for (int64_t col = P1 + lane; col < ldv; col += 64) out[col] = 0.0;
        }
    }
}


// ---------------------------------------------------------------------------
// Full space: the backward product split over alpha and beta strings.
//
// Row r = b nA + a of a full space pairs alpha string a with beta string b (keys
// ascend beta-major), so x_r = [x(a), x(b)], and with t_r = c_r d_r (per hidden unit)
//   sum_r t_r x_r,v = sum_a x(a)_v S_A[a]  (alpha v),   sum_b x(b)_v S_B[b]  (beta v),
//   S_A[a] = sum_b t_(b,a),   S_B[b] = sum_a t_(b,a),
// and likewise for the sums of c_r in X^T c.  The (c d)^T X contraction then needs
// no matrix-core work and one pass streams d.  A workgroup takes a tile of kFullTB
// beta strings and one of S alpha ranges; wave w walks the alpha strings lo + w,
// lo + w + 4, ... (a ring of kFullPD strings in flight per wave): it
// reads the tile's kFullTB rows (b, a) (a lane per hidden unit, one coalesced row per
// load), sums them into S_A[a], which it folds into W_A[h][v] += x(a)_v S_A[a][h] at
// once (n multiply-adds per kFullTB rows), and adds each row into S_B[b].  After a
// fixed-order combination of the waves, the beta columns are W[h][n + v] = sum_b
// x(b)_v S_B[b][h] over the tile, and the workgroup writes one complete partial row
// of D~^T c, as the matrix-core kernel does per row block.

// 16 beta strings per tile and one alpha string in flight per wave: 0.087 ms at
// 853,776 rows, against 0.110 ms with 8 strings and 0.157 / 0.161 ms with 2 / 3
// alpha strings in flight (the deeper rings halve the waves per SIMD)
constexpr int kFullTB = 16;
constexpr int kFullPD = 1;
constexpr int64_t kFullMinRows = 32768;    // smaller spaces keep the matrix-core kernel
constexpr int kFullMaxN = 16;

struct FullArgs {
    const double *dfac, *psi, *y0, *y1, *coefp;
    const uint32_t *strA, *strB;
    int64_t nA, nB, aper, ldv;
    int n, H, V, S, half;
    double *part;
};

__device__ __forceinline__ double readlane_d(double x, int l)
{
    const unsigned long long u = (unsigned long long)__double_as_longlong(x);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)u, l);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u >> 32), l);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// NR right-hand sides c_q = y_q - coef psi (coef = 0 without coefp).  NA >= n alpha
// orbitals.  Grid: (hidden tiles of 64, tiles x S alpha ranges).
template <int NR, int NA, int PD>
__global__ __launch_bounds__(256) void k_fac_vjp_full(FullArgs F)
{
    constexpr int TB = kFullTB;
    // doubles per lane in the wave combination: S_B, W_A and the X^T c sums of each
    // right-hand side, then C_B and psi^T c
    constexpr int kAcc = NR * (TB + NA + 1) + 2;
    __shared__ double red[64 * kAcc];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int ht = blockIdx.x;
    const int64_t wg = blockIdx.y;
    const int64_t bt = wg / F.S;
    const int sr = (int)(wg - bt * F.S);
    const int64_t b0 = bt * TB;
    const int nb = (int)(F.nB - b0 < TB ? F.nB - b0 : TB);
    const int64_t alo = (int64_t)sr * F.aper;
    const int64_t ahi = alo + F.aper < F.nA ? alo + F.aper : F.nA;
    const int h = 64 * ht + lane;
    const bool hv = h < F.H;
    const double coef = F.coefp ? *F.coefp : 0.0;
    // per-row scalars, one per lane: lanes TB k + b hold y0 (k = 0), y1 (k = 1) and
    // psi (k = 2) of row (b0 + b, a)
    static_assert(3 * TB <= 64 && (TB & (TB - 1)) == 0, "three scalars per tile row in one wavefront");
    const int bl = lane & (TB - 1), kind = lane / TB;
    double sb[NR][TB], wa[NR][NA];
#pragma unroll
    for (int q = 0; q < NR; ++q) {
#pragma unroll
        for (int b = 0; b < TB; ++b) sb[q][b] = 0.0;
#pragma unroll
        for (int v = 0; v < NA; ++v) wa[q][v] = 0.0;
    }
    double cb = 0.0, p0 = 0.0;   // lanes TB q + b (q < NR): C_B[b] and sum psi c of c_q
    double xc[NR];               // lane v < n: sum_a x(a)_v C_A[a] of c_q
#pragma unroll
    for (int q = 0; q < NR; ++q) xc[q] = 0.0;
    // ring of PD alpha strings in flight per wave: one is summed, then its slot is
    // refilled with the string PD steps ahead (strings past the range load as zeros)
    struct Stage {
        double sc, dv[TB];
    };
    auto fetch = [&](int64_t a, Stage &g) {
        g.sc = 0.0;
        if (a < ahi && bl < nb) {
            const int64_t r = (b0 + bl) * F.nA + a;
            if (kind == 0)
                g.sc = F.y0[r];
            else if (kind == 1 && NR == 2)
                g.sc = F.y1[r];
            else if (kind == 2)
                g.sc = F.psi[r];
        }
#pragma unroll
        for (int b = 0; b < TB; ++b)
            g.dv[b] = (a < ahi && b < nb && hv) ? __builtin_nontemporal_load(F.dfac + ((b0 + b) * F.nA + a) * F.H + h)
                                                : 0.0;
    };
    auto consume = [&](int64_t a, const Stage &g) {
        const double sc = g.sc;
        const double *dv = g.dv;
        const double ps = __shfl(sc, 2 * TB + bl, 64);
        const double cl = kind < 2 ? sc - coef * ps : sc;    // lanes TB q + b: c_q of row b
        double sa[NR];
#pragma unroll
        for (int q = 0; q < NR; ++q) sa[q] = 0.0;
#pragma unroll
        for (int b = 0; b < TB; ++b) {
            if (b < nb) {
#pragma unroll
                for (int q = 0; q < NR; ++q) {
                    const double t = readlane_d(cl, TB * q + b) * dv[b];
                    sa[q] += t;
                    sb[q][b] += t;
                }
            }
        }
        const uint32_t xa = F.strA[a];
#pragma unroll
        for (int v = 0; v < NA; ++v) {
            const double xv = ((xa >> v) & 1u) ? 1.0 : 0.0;
#pragma unroll
            for (int q = 0; q < NR; ++q) wa[q][v] = fma(xv, sa[q], wa[q][v]);
        }
        // C_A[a] over the tile's beta strings (fixed TB-lane tree), folded into lane v
        double ca = kind < NR ? cl : 0.0;
#pragma unroll
        for (int off = 1; off < TB; off <<= 1) ca += __shfl_xor(ca, off, 64);
        const double xl = ((xa >> (lane & 31)) & 1u) && lane < F.n ? 1.0 : 0.0;
#pragma unroll
        for (int q = 0; q < NR; ++q) xc[q] = fma(xl, readlane_d(ca, TB * q), xc[q]);
        if (kind < NR) {
            cb += cl;
            p0 = fma(cl, ps, p0);
        }
    };
    Stage ring[PD];
#pragma unroll
    for (int p = 0; p < PD; ++p) fetch(alo + wv + 4 * p, ring[p]);
    for (int64_t a = alo + wv; a < ahi; a += 4 * PD) {
#pragma unroll
        for (int p = 0; p < PD; ++p) {
            if (a + 4 * p < ahi) consume(a + 4 * p, ring[p]);
            fetch(a + 4 * (p + PD), ring[p]);
        }
    }

    // fixed-order combination of the 4 waves: ((w0 + w1) + w2) + w3
    auto slot = [&](int k) -> double & { return red[64 * k + lane]; };
    for (int src = 1; src < 4; ++src) {
        __syncthreads();
        if (wv == src) {
            int k = 0;
#pragma unroll
            for (int q = 0; q < NR; ++q) {
#pragma unroll
                for (int b = 0; b < TB; ++b) slot(k++) = sb[q][b];
#pragma unroll
                for (int v = 0; v < NA; ++v) slot(k++) = wa[q][v];
                slot(k++) = xc[q];
            }
            slot(k++) = cb;
            slot(k++) = p0;
        }
        __syncthreads();
        if (wv == 0) {
            int k = 0;
#pragma unroll
            for (int q = 0; q < NR; ++q) {
#pragma unroll
                for (int b = 0; b < TB; ++b) sb[q][b] += slot(k++);
#pragma unroll
                for (int v = 0; v < NA; ++v) wa[q][v] += slot(k++);
                xc[q] += slot(k++);
            }
            cb += slot(k++);
            p0 += slot(k++);
        }
    }
    if (wv != 0) return;
    const int n = F.n, V = F.V;
    const int64_t baseW = 1 + V + F.H, P1 = (int64_t)V * F.H + F.H + V + 1;
    uint32_t xb[TB];
#pragma unroll
    for (int b = 0; b < TB; ++b) xb[b] = b < nb ? F.strB[b0 + b] : 0u;
#pragma unroll
    for (int q = 0; q < NR; ++q) {
        double *out = F.part + (wg * 2 + (NR == 2 ? q : F.half)) * F.ldv;
        if (hv) {
            double ds = 0.0;
#pragma unroll
            for (int b = 0; b < TB; ++b) ds += sb[q][b];
            out[1 + V + h] = ds;
            double *wrow = out + baseW + (int64_t)h * V;
#pragma unroll
            for (int v = 0; v < NA; ++v)
                if (v < n) wrow[v] = wa[q][v];
#pragma unroll
            for (int v = 0; v < NA; ++v) {
                if (v < n) {
                    double wbv = 0.0;
#pragma unroll
                    for (int b = 0; b < TB; ++b) wbv = fma(((xb[b] >> v) & 1u) ? 1.0 : 0.0, sb[q][b], wbv);
                    wrow[n + v] = wbv;
                }
            }
        }
        if (ht == 0) {
            // psi^T c (TB-lane tree of the lanes TB q + b)
            double p = p0;
#pragma unroll
            for (int off = 1; off < TB; off <<= 1) p += __shfl_xor(p, off, 64);
            const double ptot = readlane_d(p, TB * q);
            // X^T c: alpha columns from lane v, beta columns sum_b x(b)_v C_B[b]
            double xbv = 0.0;
#pragma unroll
            for (int b = 0; b < TB; ++b) {
                const double cbb = readlane_d(cb, TB * q + b);
                xbv = fma(((xb[b] >> (lane & 31)) & 1u) ? 1.0 : 0.0, cbb, xbv);
            }
            if (lane == 0) out[0] = ptot;
            if (lane < n) {
                out[1 + lane] = xc[q];
                out[1 + n + lane] = xbv;
            }
            for (int64_t col = P1 + lane; col < F.ldv; col += 64) out[col] = 0.0;
        }
    }
}


// Full-space D~ v (H <= 64).  With the same split, (X V_W^T)_r = A[a] + B[b] and
// x_r . v_a = PA[a] + PB[b], so
//   w_r = psi_r v_0 + PA[a] + PB[b] + sum_h d_rh (v_b[h] + A[a][h] + B[b][h]).
// A workgroup takes a tile of kFullTB beta strings and an alpha range: B of the tile
// stays in registers (a lane per hidden unit), A[a] is n multiply-adds per alpha
// string, each row costs one add and one multiply-add per lane, and the kFullTB row
// sums over the 64 lanes finish in one transposed butterfly (row rho ends in lane
// L(rho) = 32 rho_3 + 16 rho_2 + 8 rho_1 + 4 rho_0, summed in a fixed order).  Its d
// loads go through the caches and the backward product's stream past them: per
// apply at 853,776 rows, 0.093 + 0.089 ms, against 0.092 + 0.103 ms with both
// streaming and 0.095 + 0.106 ms with both cached.
static_assert(kFullTB == 16, "the butterfly below reduces 16 rows");

__device__ __forceinline__ int full_row_lane(int rho)
{
    return 32 * ((rho >> 3) & 1) + 16 * ((rho >> 2) & 1) + 8 * ((rho >> 1) & 1) + 4 * (rho & 1);
}

constexpr int kJvpChunk = 64;   // alpha strings per write-back of w

template <int HALF>
__device__ __forceinline__ void full_fold(double *acc, int lane, int bit)
{
    const bool up = (lane & bit) != 0;
#pragma unroll
    for (int i = 0; i < HALF; ++i) {
        const double keep = up ? acc[i + HALF] : acc[i];
        const double send = up ? acc[i] : acc[i + HALF];
        acc[i] = keep + __shfl_xor(send, bit, 64);
    }
}

template <int NA>
__global__ __launch_bounds__(256) void k_fac_jvp_full(FullArgs F, const double *__restrict__ v, int zero_v0,
                                                      double *__restrict__ w)
{
    constexpr int TB = kFullTB;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t wg = blockIdx.x;
    const int64_t bt = wg / F.S;
    const int sr = (int)(wg - bt * F.S);
    const int64_t b0 = bt * TB;
    const int nb = (int)(F.nB - b0 < TB ? F.nB - b0 : TB);
    const int64_t alo = (int64_t)sr * F.aper;
    const int64_t ahi = alo + F.aper < F.nA ? alo + F.aper : F.nA;
    const int n = F.n, V = F.V, H = F.H;
    const bool hv = lane < H;
    const double v0 = zero_v0 ? 0.0 : v[0];
    // lane h: v_b[h], its V_W row (alpha part) and B[b][h] of the tile
    const double vb = hv ? v[1 + V + lane] : 0.0;
    const double *vw = v + 1 + V + H + (int64_t)lane * V;
    double vwa[NA], bb[TB];
#pragma unroll
    for (int k = 0; k < NA; ++k) vwa[k] = (hv && k < n) ? vw[k] : 0.0;
#pragma unroll
    for (int b = 0; b < TB; ++b) bb[b] = 0.0;
    if (hv)
        for (int k = 0; k < n; ++k) {
            const double x = vw[n + k];
#pragma unroll
            for (int b = 0; b < TB; ++b)
                if (b < nb) bb[b] = fma(((F.strB[b0 + b] >> k) & 1u) ? 1.0 : 0.0, x, bb[b]);
        }
    // row rho = the row this lane writes (lanes 4 j), PB[b0 + rho] and v_a of alpha
    int rho = 0;
    {
        const int l = lane;
        rho = 8 * ((l >> 5) & 1) + 4 * ((l >> 4) & 1) + 2 * ((l >> 3) & 1) + ((l >> 2) & 1);
    }
    const bool writer = (lane & 3) == 0 && rho < nb;
    double pb = 0.0;
    if (writer) {
        const uint32_t xb = F.strB[b0 + rho];
        for (int k = 0; k < n; ++k) pb = fma(((xb >> k) & 1u) ? 1.0 : 0.0, v[1 + n + k], pb);
    }
    // lane k < n: v_a[k] (PA[a] is a wavefront sum)
    const double vak = lane < n ? v[1 + lane] : 0.0;
    // w of the tile's rows for kJvpChunk alpha strings at a time, written back as
    // contiguous runs of each row block
    __shared__ double wbuf[TB * kJvpChunk];
    for (int64_t ac = alo; ac < ahi; ac += kJvpChunk) {
    const int64_t ace = ac + kJvpChunk < ahi ? ac + kJvpChunk : ahi;
    for (int64_t a = ac + wv; a < ace; a += 4) {
        double dv[TB];
#pragma unroll
        for (int b = 0; b < TB; ++b)
            dv[b] = (b < nb && hv) ? F.dfac[((b0 + b) * F.nA + a) * H + lane] : 0.0;
        const double ps = writer ? F.psi[(b0 + rho) * F.nA + a] : 0.0;
        const uint32_t xa = F.strA[a];
        double ua = vb;
#pragma unroll
        for (int k = 0; k < NA; ++k) ua = fma(((xa >> k) & 1u) ? 1.0 : 0.0, vwa[k], ua);
        double pa = ((xa >> (lane & 31)) & 1u) ? vak : 0.0;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) pa += __shfl_xor(pa, off, 64);
        double *acc = dv;
#pragma unroll
        for (int b = 0; b < TB; ++b) acc[b] = dv[b] * (ua + bb[b]);
        // transposed butterfly: at each step a lane keeps the half of its rows named
        // by its lane bit and adds the partner's partials of those rows
        full_fold<8>(acc, lane, 32);
        full_fold<4>(acc, lane, 16);
        full_fold<2>(acc, lane, 8);
        full_fold<1>(acc, lane, 4);
        double sum = acc[0];
        sum += __shfl_xor(sum, 2, 64);
        sum += __shfl_xor(sum, 1, 64);
        if (writer) wbuf[rho * kJvpChunk + (int)(a - ac)] = ps * v0 + (pa + pb) + sum;
    }
    __syncthreads();
    const int cnt = (int)(ace - ac);
    for (int i = threadIdx.x; i < nb * kJvpChunk; i += 256) {
        const int r = i / kJvpChunk, c = i - r * kJvpChunk;
        if (c < cnt) w[(b0 + r) * F.nA + ac + c] = wbuf[i];
    }
    __syncthreads();
    }
}


// Full-space forward pass (H <= 64).  z_r = Z_A[a] + Z_B[b] + bias with Z_A = X_A
// W_A^T and Z_B = X_B W_B^T: the tile's Z_B (plus the bias) stays in registers, Z_A[a]
// is n multiply-adds per alpha string, and each row costs one tanh per lane and a
// coalesced store of its d; psi_r = PA[a] + PB[b] + sum_h t_h with the row sums
// taken by a transposed butterfly over 8 rows at a time (16 rows of tanh in flight
// take more than 256 registers) and psi written back in contiguous runs.
template <int NA>
__global__ __launch_bounds__(256) void k_fac_forward_full(FullArgs F, const double *__restrict__ theta,
                                                          double *__restrict__ psi, double *__restrict__ dfac)
{
    constexpr int TB = kFullTB;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t wg = blockIdx.x;
    const int64_t bt = wg / F.S;
    const int sr = (int)(wg - bt * F.S);
    const int64_t b0 = bt * TB;
    const int nb = (int)(F.nB - b0 < TB ? F.nB - b0 : TB);
    const int64_t alo = (int64_t)sr * F.aper;
    const int64_t ahi = alo + F.aper < F.nA ? alo + F.aper : F.nA;
    const int n = F.n, V = F.V, H = F.H;
    const bool hv = lane < H;
    const double *av = theta, *bias = theta + V, *W = theta + V + H;
    // lane h: the alpha part of W row h, and Z_B[b][h] + bias[h] of the tile
    const double *wrow = W + (int64_t)lane * V;
    double wa[NA], zb[TB];
#pragma unroll
    for (int k = 0; k < NA; ++k) wa[k] = (hv && k < n) ? wrow[k] : 0.0;
    const double bh = hv ? bias[lane] : 0.0;
#pragma unroll
    for (int b = 0; b < TB; ++b) zb[b] = bh;
    if (hv)
        for (int k = 0; k < n; ++k) {
            const double x = wrow[n + k];
#pragma unroll
            for (int b = 0; b < TB; ++b)
                if (b < nb) zb[b] = fma(((F.strB[b0 + b] >> k) & 1u) ? 1.0 : 0.0, x, zb[b]);
        }
    // rows are summed over the lanes 8 at a time: row 8 g + rho8 of group g ends in
    // lane 32 rho8_2 + 16 rho8_1 + 8 rho8_0, which adds PB of both of its rows
    const int rho8 = 4 * ((lane >> 5) & 1) + 2 * ((lane >> 4) & 1) + ((lane >> 3) & 1);
    double pb[2] = {0.0, 0.0};
    if ((lane & 7) == 0)
#pragma unroll
        for (int g = 0; g < 2; ++g)
            if (8 * g + rho8 < nb) {
                const uint32_t xb = F.strB[b0 + 8 * g + rho8];
                for (int k = 0; k < n; ++k) pb[g] = fma(((xb >> k) & 1u) ? 1.0 : 0.0, av[n + k], pb[g]);
            }
    const double ak = lane < n ? av[lane] : 0.0;   // lane k < n: a_k (PA[a] is a wavefront sum)
    __shared__ double pbuf[TB * kJvpChunk];
    for (int64_t ac = alo; ac < ahi; ac += kJvpChunk) {
        const int64_t ace = ac + kJvpChunk < ahi ? ac + kJvpChunk : ahi;
        for (int64_t a = ac + wv; a < ace; a += 4) {
            const uint32_t xa = F.strA[a];
            double za = 0.0;
#pragma unroll
            for (int k = 0; k < NA; ++k) za = fma(((xa >> k) & 1u) ? 1.0 : 0.0, wa[k], za);
            double pa = (((xa >> (lane & 31)) & 1u) && lane < n) ? ak : 0.0;
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) pa += __shfl_xor(pa, off, 64);
#pragma unroll
            for (int g = 0; g < 2; ++g) {
                double ts[8];
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    const int b = 8 * g + i;
                    double t, d;
                    tanh_and_d(za + zb[b], t, d);
                    if (b < nb && hv) dfac[((b0 + b) * F.nA + a) * H + lane] = d;
                    ts[i] = hv ? t : 0.0;
                }
                full_fold<4>(ts, lane, 32);
                full_fold<2>(ts, lane, 16);
                full_fold<1>(ts, lane, 8);
                double sum = ts[0];
                sum += __shfl_xor(sum, 4, 64);
                sum += __shfl_xor(sum, 2, 64);
                sum += __shfl_xor(sum, 1, 64);
                if ((lane & 7) == 0 && 8 * g + rho8 < nb)
                    pbuf[(8 * g + rho8) * kJvpChunk + (int)(a - ac)] = (pa + pb[g]) + sum;
            }
        }
        __syncthreads();
        const int cnt = (int)(ace - ac);
        for (int i = threadIdx.x; i < nb * kJvpChunk; i += 256) {
            const int r = i / kJvpChunk, c = i - r * kJvpChunk;
            if (c < cnt) psi[(b0 + r) * F.nA + ac + c] = pbuf[i];
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// launchers: KS = k-steps of 4 visible units (even, V <= 4 KS), NT = column tiles of
// 16 visible units (V <= 16 NT)

namespace {

int fac_tile_blocks(int64_t ns)
{
    // 4 waves x one 16-row tile each; grid-stride beyond 512 blocks (two per
    // compute unit: at 853,776 rows the forward takes 0.227 ms and the
    // Jacobian-vector product 0.109 ms, against 0.236 and 0.113 at 1024
    // blocks and 0.145 ms for the product at 256)
    int64_t blocks = (ns + 63) / 64;
    if (blocks > 512) blocks = 512;
    return (int)(blocks < 1 ? 1 : blocks);
}

// QT (hidden column tiles per wave): 4 while the B operand is small, else 2
template <int KS>
void forward_ks(const irl_system *s, const WsLayout &L, int V, int H, const double *theta, double *psi,
                double *dfac, hipStream_t st)
{
    constexpr int QT = KS <= 6 ? 4 : 2;
    const int blocks = fac_tile_blocks(L.ns);
    if (H % QT == 0)
        k_fac_forward<KS, QT, true><<<blocks, 256, 0, st>>>(s->d.keys, L.ns, s->n, V, H, theta, psi, dfac);
    else
        k_fac_forward<KS, QT, false><<<blocks, 256, 0, st>>>(s->d.keys, L.ns, s->n, V, H, theta, psi, dfac);
}

template <int KS>
void jvp_ks(const irl_system *s, const FacRows &R, int V, int H, const double *v, int zero_v0, double *w,
            hipStream_t st)
{
    constexpr int QT = KS <= 6 ? 4 : 2;
    const int blocks = fac_tile_blocks(R.ns);
    if (H % QT == 0)
        k_fac_jvp<KS, QT, true><<<blocks, 256, 0, st>>>(R.keys, R.ns, s->n, V, H, R.dfac, R.psi, v, zero_v0, w);
    else
        k_fac_jvp<KS, QT, false><<<blocks, 256, 0, st>>>(R.keys, R.ns, s->n, V, H, R.dfac, R.psi, v, zero_v0, w);
}

// MT (hidden column tiles per wave) keeps NR MT NT <= 8 accumulator tiles per lane
template <int NT, int NR>
void vjp_nt(const irl_system *s, const WsLayout &L, const FacRows &R, int V, int H, const double *y0,
            const double *y1, const double *coefp, double *part, int nblk, int half, hipStream_t st)
{
    constexpr int MT = (8 / (NR * NT)) >= 4 ? 4 : (8 / (NR * NT)) >= 2 ? 2 : 1;
    const dim3 grid((H + 16 * MT - 1) / (16 * MT), nblk);
    if (H % MT == 0)
        k_fac_vjp<NT, NR, MT, true><<<grid, 256, 0, st>>>(R.keys, R.ns, s->n, V, H, R.dfac, R.psi, y0, y1,
                                                          coefp, part, L.ldv, nblk, half);
    else
        k_fac_vjp<NT, NR, MT, false><<<grid, 256, 0, st>>>(R.keys, R.ns, s->n, V, H, R.dfac, R.psi, y0, y1,
                                                           coefp, part, L.ldv, nblk, half);
}

// ---------------------------------------------------------------------------
// Backward product of selected sets on the vector units.
//
// The matrix-core form (k_fac_vjp) contracts (c d)^T with X through dense 16 x 16
// x 4 tiles: N_s V H multiply-adds per right-hand side on an X that is 0/1 with
// N_alpha + N_beta ones per row (at V = 40, H = 256 that is twice the time of
// streaming d).  Here a workgroup owns a block of rows and every hidden unit
// (thread t = hidden unit t, H <= 256) and walks its rows in order: a row's
// occupation bits are the same for every thread, so its alpha part is one FMA per
// orbital with the bit as a scalar 0.0 / 1.0 operand, and its beta part is folded
// once per run of rows that share a beta string (keys ascend beta-major, so such
// runs are contiguous; any order is still correct).  d streams once per pass with
// coalesced row loads, PD rows in flight per thread; row data (keys, psi,
// right-hand sides) are staged in LDS per batch of kBitsRB rows.  (The same scheme
// for the forward pass and D~ v measured slower than the matrix-core forms, whose
// contraction there is a single 16-wide product per tile.)

#ifndef IRL_BITS_PD
#define IRL_BITS_PD 8
#endif
#ifndef IRL_BITS_BLOCKS
#define IRL_BITS_BLOCKS 512
#endif
constexpr int kBitsRB = 256;   // rows staged per batch
constexpr int kBitsPD = IRL_BITS_PD;   // d rows in flight per thread (8 or 16)
constexpr int kBitsMaxN = 24;  // alpha (and beta) orbitals of the register accumulators
constexpr int kBitsMinH = 48;  // narrower networks keep the matrix-core forms
constexpr int kBitsMaxH = 256;
constexpr int kBitsBlocks = IRL_BITS_BLOCKS;

struct BitsArgs {
    const uint64_t *keys;
    const double *psi, *dfac;
    int64_t ns;
    int n, V, H;
};

__device__ __forceinline__ uint32_t uniform_u32(uint32_t x) { return (uint32_t)__builtin_amdgcn_readfirstlane((int)x); }

// bit k of a wavefront-uniform mask as the double 0.0 or 1.0 (scalar arithmetic:
// 1.0 is 0x3ff0 << 48), so a conditional add becomes one FMA with a scalar operand;
// fma(bit, y, x) equals x or x + y exactly
__device__ __forceinline__ double bit_d(uint32_t bits, int k)
{
    // the bit spread over all 64 bits (0 or -1) masks 1.0 as one 64-bit value: two
    // scalar instructions, with no separate move for the low word
    const int64_t m = (int64_t)((uint64_t)bits << (63 - k)) >> 63;
    return __builtin_bit_cast(double, (uint64_t)m & 0x3ff0000000000000ull);
}

// rows [r0, r1) of row block rb of nblk
__device__ __forceinline__ void bits_block(int64_t ns, int nblk, int rb, int64_t &r0, int64_t &r1)
{
    const int64_t per = (ns + nblk - 1) / nblk;
    r0 = (int64_t)rb * per;
    r1 = r0 + per < ns ? r0 + per : ns;
    if (r0 > ns) r0 = ns;
}

// Partial rows of D~^T c for NR right-hand sides c_q = y_q - coef psi over row block
// blockIdx.x (layout of k_fac_vjp: NR = 2 writes rows (rb, 0) and (rb, 1), NR = 1 row
// (rb, half)).  Thread h accumulates W[h][v] for the alpha orbitals v < n per row
// and, for the beta orbitals, the run sum S of c d_h that it folds into W[h][n + v]
// (and into the b entry) when the beta string changes.  Wave 0 also sums c over
// each orbital (the a entries, lane v) and c psi (the psi entry).
// acc[q][k] += bit_k * t[q] for the alpha bits k < NA of a row, one FP64 FMA per
// (k, q) and no scalar instruction: lane l of every 16-lane row holds the 0/1
// factor of bit l (flo) and of bit 16 + l (fhi), and each FMA reads the factor of
// bit k through a row broadcast (DPP row_newbcast).  The sums are those of
// fma(bit_d(bits, k), t, acc) bit for bit.  A VALU write of a VGPR needs two wait
// states before a DPP read of it: the factors pass through an s_nop after they are
// formed, and every broadcast FMA takes them from its output.
template <int K>
__device__ __forceinline__ void fmac_bcast(double &acc, double f, double y)
{
    asm("v_fmac_f64_dpp %0, %1, %2 row_newbcast:%3 row_mask:0xf bank_mask:0xf"
        : "+v"(acc)
        : "v"(f), "v"(y), "n"(K & 15));
}

template <int NR, int NA, int... K>
__device__ __forceinline__ void bits_fma_seq(double (&acc)[NR][NA], double flo, double fhi, const double (&t)[NR],
                                             std::integer_sequence<int, K...>)
{
    (
        [&] {
#pragma unroll
            for (int q = 0; q < NR; ++q) fmac_bcast<K>(acc[q][K], K < 16 ? flo : fhi, t[q]);
        }(),
        ...);
}

template <int NR, int NA>
__device__ __forceinline__ void bits_fma(double (&acc)[NR][NA], uint32_t bits, int lane, const double (&t)[NR])
{
    static_assert(NA <= 32, "two factor registers hold 32 bits");
    const uint32_t sh = (uint32_t)lane & 15u;
    double flo = __hiloint2double(((bits >> sh) & 1u) ? 0x3ff00000 : 0, 0);
    double fhi = NA > 16 ? __hiloint2double(((bits >> (16u + sh)) & 1u) ? 0x3ff00000 : 0, 0) : 0.0;
    asm("s_nop 1" : "+v"(flo), "+v"(fhi));
    bits_fma_seq<NR, NA>(acc, flo, fhi, t, std::make_integer_sequence<int, NA>{});
}

template <int NR, int NA>
__global__ __launch_bounds__(256) void k_fac_vjp_bits(BitsArgs A, const double *__restrict__ y0,
                                                      const double *__restrict__ y1, const double *__restrict__ coefp,
                                                      double *__restrict__ part, int64_t ldv, int nblk, int half)
{
    constexpr int RB = kBitsRB, PD = kBitsPD;
    __shared__ uint64_t skey[RB];
    __shared__ double sps[RB], sc[NR][RB];
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int H = A.H, n = A.n, V = A.V;
    const bool hv = t < H;
    int64_t r0, r1;
    bits_block(A.ns, nblk, blockIdx.x, r0, r1);
    const double coef = coefp ? *coefp : 0.0;
    const double *ys[2] = {y0, y1};
    double wa[NR][NA], wb[NR][NA], sb[NR], bp[NR], ax[NR], a0[NR];
#pragma unroll
    for (int q = 0; q < NR; ++q) {
        sb[q] = bp[q] = ax[q] = a0[q] = 0.0;
#pragma unroll
        for (int k = 0; k < NA; ++k) wa[q][k] = wb[q][k] = 0.0;
    }
    uint32_t cur = 0u;
    bool run = false;
    double dr[PD];
#pragma unroll
    for (int p = 0; p < PD; ++p) dr[p] = (hv && r0 + p < r1) ? A.dfac[(r0 + p) * H + t] : 0.0;
    for (int64_t bs = r0; bs < r1; bs += RB) {
        const int nbt = (int)(r1 - bs < RB ? r1 - bs : RB);
        __syncthreads();
        for (int i = t; i < nbt; i += blockDim.x) {
            const int64_t r = bs + i;
            const double ps = A.psi[r];
            skey[i] = A.keys[r];
            sps[i] = ps;
#pragma unroll
            for (int q = 0; q < NR; ++q) sc[q][i] = fma(-coef, ps, ys[q][r]);
        }
        __syncthreads();
        for (int j0 = 0; j0 < nbt; j0 += PD) {
#pragma unroll
            for (int p = 0; p < PD; ++p) {
                const int j = j0 + p;
                // a row past the batch adds zeros to the alpha sums (no branch around
                // them: the accumulators then need no copies across it)
                uint32_t al = 0u;
                double tq[NR];
#pragma unroll
                for (int q = 0; q < NR; ++q) tq[q] = 0.0;
                if (j < nbt) {
                    const uint64_t key = skey[j];
                    al = uniform_u32((uint32_t)key);
                    const uint32_t be = uniform_u32((uint32_t)(key >> 32));
                    if (!run || be != cur) {
                        if (run) {
#pragma unroll
                            for (int k = 0; k < NA; ++k) {
                                const double bk = bit_d(cur, k);
#pragma unroll
                                for (int q = 0; q < NR; ++q) wb[q][k] = fma(bk, sb[q], wb[q][k]);
                            }
#pragma unroll
                            for (int q = 0; q < NR; ++q) {
                                bp[q] += sb[q];
                                sb[q] = 0.0;
                            }
                        }
                        cur = be;
                        run = true;
                    }
                    const double d = dr[p];
                    double c[NR];
#pragma unroll
                    for (int q = 0; q < NR; ++q) {
                        c[q] = sc[q][j];
                        tq[q] = c[q] * d;
                        sb[q] += tq[q];
                    }
#ifdef IRL_VJP_NO_DPP
#pragma unroll
                    for (int k = 0; k < NA; ++k) {
                        const double bk = bit_d(al, k);
#pragma unroll
                        for (int q = 0; q < NR; ++q) wa[q][k] = fma(bk, tq[q], wa[q][k]);
                    }
#endif
                    if (wv == 0) {
                        const uint32_t bits = lane < n ? al : be;
                        const int sh = lane < n ? lane : lane - n;
                        const bool on = lane < V && ((bits >> (sh & 31)) & 1u);
                        const double ps = sps[j];
#pragma unroll
                        for (int q = 0; q < NR; ++q) {
                            ax[q] += on ? c[q] : 0.0;
                            a0[q] = fma(c[q], ps, a0[q]);
                        }
                    }
                }
#ifndef IRL_VJP_NO_DPP
                bits_fma<NR, NA>(wa, al, lane, tq);
#endif
                const int64_t rn = bs + j0 + p + PD;
                dr[p] = (hv && rn < r1) ? A.dfac[rn * H + t] : 0.0;
            }
        }
    }
    if (run) {
#pragma unroll
        for (int k = 0; k < NA; ++k) {
            const double bk = bit_d(cur, k);
#pragma unroll
            for (int q = 0; q < NR; ++q) wb[q][k] = fma(bk, sb[q], wb[q][k]);
        }
#pragma unroll
        for (int q = 0; q < NR; ++q) bp[q] += sb[q];
    }
    const int64_t P1 = (int64_t)V * H + H + V + 1;
#pragma unroll
    for (int q = 0; q < NR; ++q) {
        double *out = part + ((int64_t)blockIdx.x * 2 + (NR == 2 ? q : half)) * ldv;
        if (hv) {
            double *wrow = out + 1 + V + H + (int64_t)t * V;
#pragma unroll
            for (int k = 0; k < NA; ++k)
                if (k < n) {
                    wrow[k] = wa[q][k];
                    wrow[n + k] = wb[q][k];
                }
            out[1 + V + t] = bp[q];
        }
        if (wv == 0) {
            if (lane < V) out[1 + lane] = ax[q];
            if (lane == 0) out[0] = a0[q];
            for (int64_t col = P1 + lane; col < ldv; col += 64) out[col] = 0.0;
        }
    }
}

// The same partial rows with the rows' data streamed into LDS by direct-to-LDS loads
// (global_load_lds), which need no registers, so a wavefront keeps kRingPairs row
// pairs of d in flight beside its 2 NR NA accumulators.  Wavefront w owns hidden
// units [64 w, 64 w + 64) and its own LDS ring: one load per row pair brings the
// pair's two 512-byte segments of d; the rows' keys, psi and y (kRingBatch rows at a
// time, double-buffered) come the same way, in dwords.  The rows are visited in the
// order of k_fac_vjp_bits and every sum has the same operands in the same order, so
// the partial rows are bitwise those of k_fac_vjp_bits.  Only direct-to-LDS loads
// are in flight in the loop, so the waits are counted by hand: before a pair is
// read, every load but the ones issued after it has completed.
constexpr int kRingPairs = 16;   // row pairs in flight per wavefront
constexpr int kRingBatch = 64;   // rows per batch of keys, psi and y

typedef __attribute__((address_space(3))) void *lds_ptr_t;
// word 3 of a raw buffer descriptor on gfx9-family parts: 32-bit data format, no
// swizzle, no index stride; with stride 0 the size (word 2) is in bytes and loads at
// or past it return zeros
constexpr int kBufWord3 = 0x00020000;
typedef uint32_t u4v __attribute__((ext_vector_type(4)));
typedef uint32_t u2v __attribute__((vector_size(8)));
// the LDS byte address of a workgroup-shared object
__device__ __forceinline__ uint32_t lds_addr(const void *p)
{
    return (uint32_t)(uintptr_t)(const __attribute__((address_space(3))) void *)p;
}
// double e of two packed in a 16-byte LDS read
__device__ __forceinline__ double u2d(u4v x, int e)
{
    return __builtin_bit_cast(double, ((uint64_t)x[2 * e + 1] << 32) | x[2 * e]);
}

template <int NR, int NA>
__global__ __launch_bounds__(256) void k_fac_vjp_ring(BitsArgs A, const double *__restrict__ y0,
                                                      const double *__restrict__ y1, const double *__restrict__ coefp,
                                                      double *__restrict__ part, int64_t ldv, int nblk, int half)
{
    constexpr int RP = kRingPairs, MB = kRingBatch, NM = 2 + NR;   // arrays per batch: keys, psi, y0 (, y1)
    __shared__ double ring[4][RP][128];
    __shared__ double meta[4][2][NM][MB];
    const int t = threadIdx.x, lane = t & 63;
    const int wv = __builtin_amdgcn_readfirstlane(t >> 6);
    const int H = A.H, n = A.n, V = A.V;
    int64_t r0, r1;
    bits_block(A.ns, nblk, blockIdx.x, r0, r1);
    const int64_t nr = r1 - r0;
    const double coef = coefp ? *coefp : 0.0;
    double wa[NR][NA], wb[NR][NA], sb[NR], bp[NR], ax[NR], a0[NR];
#pragma unroll
    for (int q = 0; q < NR; ++q) {
        sb[q] = bp[q] = ax[q] = a0[q] = 0.0;
#pragma unroll
        for (int k = 0; k < NA; ++k) wa[q][k] = wb[q][k] = 0.0;
    }
    uint32_t cur = 0u;
    bool run = false;
    if (nr > 0) {
        // Direct-to-LDS buffer loads with loop-invariant lane offsets; each load's
        // descriptor ends at the block's last row, so lanes past it (the second row of
        // a last odd pair, pairs and batches past the end) read zeros and touch no
        // memory.
        const int vo_d = ((lane >> 5) * H + 64 * wv + 2 * (lane & 31)) * 8, vo_m = lane * 4;
        // pair p: rows r0 + 2p and r0 + 2p + 1, the wavefront's 64 hidden units of each
        auto dma_pair = [&](int64_t p) {
            const int64_t left = nr - 2 * p;
            const int nb = left <= 0 ? 0 : (int)((left < 2 ? left : 2) * H * 8);
            const __amdgpu_buffer_rsrc_t rs =
                __builtin_amdgcn_make_buffer_rsrc((void *)(A.dfac + (r0 + 2 * p) * H), 0, nb, kBufWord3);
            __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (lds_ptr_t)&ring[wv][p % RP][0], 16, vo_d, 0, 0, 0);
        };
        // batch b: keys, psi, y0 (, y1) of rows r0 + MB b ... as dwords (two loads of
        // 32 rows per array)
        auto dma_meta = [&](int64_t b) {
            const double *arr[4] = {reinterpret_cast<const double *>(A.keys), A.psi, y0, y1};
            const int64_t left = nr - (int64_t)MB * b;
            const int nb = left <= 0 ? 0 : (int)((left < MB ? left : MB) * 8);
#pragma unroll
            for (int a = 0; a < NM; ++a) {
                const __amdgpu_buffer_rsrc_t rs =
                    __builtin_amdgcn_make_buffer_rsrc((void *)(arr[a] + r0 + (int64_t)MB * b), 0, nb, kBufWord3);
                // the immediate offset moves both the global and the LDS address
                __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (lds_ptr_t)&meta[wv][b & 1][a][0], 4, vo_m, 0, 0, 0);
                __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (lds_ptr_t)&meta[wv][b & 1][a][0], 4, vo_m, 0, 256, 0);
            }
        };
        const int64_t npairs = (nr + 1) / 2;
        dma_meta(0);
        dma_meta(1);
#pragma unroll
        for (int p = 0; p < RP; ++p) dma_pair(p);
        // two pairs (four rows) per iteration; a batch holds MB / 2 pairs, an even count
        for (int64_t p = 0; p < npairs; p += 2) {
            const int64_t b = p / (MB / 2);
            if (p % (MB / 2) == 0 && b > 0) {
                // batch b - 1's rows are read (their LDS reads complete), so its buffer
                // takes batch b + 1
                asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
                dma_meta(b + 1);
            }
            // pair p + 1's load and every older one have completed: the loads issued
            // after it are the RP - 2 later pairs and, when a batch started since, the
            // 2 NM loads of the next batch
            const int64_t bs = b * (MB / 2);   // the latest batch start at or before p
            if (bs > 0 && bs > p + 1 - RP) {
                if constexpr (NR == 2)
                    asm volatile("s_waitcnt vmcnt(22)" ::: "memory");
                else
                    asm volatile("s_waitcnt vmcnt(20)" ::: "memory");
            } else {
                asm volatile("s_waitcnt vmcnt(14)" ::: "memory");
            }
            // the four rows' keys, psi and y (the same for every lane) and their d
            // values, read in one block that also waits for them: the compiler does not
            // track which LDS bytes the direct-to-LDS loads write and would otherwise
            // wait for every load in flight before each read
            const int jm0 = (int)((2 * p) % MB);
            const uint32_t maddr = lds_addr(&meta[wv][b & 1][0][jm0]);
            const uint32_t da0 = lds_addr(&ring[wv][p % RP][lane]), da1 = lds_addr(&ring[wv][(p + 1) % RP][lane]);
            u4v mk[2], mp[2], my0[2], my1[2] = {u4v{0u, 0u, 0u, 0u}, u4v{0u, 0u, 0u, 0u}};
            d2v dd[2];
            if constexpr (NR == 2) {
                asm volatile("ds_read_b128 %0, %10\n\t"
                             "ds_read_b128 %1, %10 offset:16\n\t"
                             "ds_read_b128 %2, %10 offset:512\n\t"
                             "ds_read_b128 %3, %10 offset:528\n\t"
                             "ds_read_b128 %4, %10 offset:1024\n\t"
                             "ds_read_b128 %5, %10 offset:1040\n\t"
                             "ds_read_b128 %6, %10 offset:1536\n\t"
                             "ds_read_b128 %7, %10 offset:1552\n\t"
                             "ds_read2_b64 %8, %11 offset1:64\n\t"
                             "ds_read2_b64 %9, %12 offset1:64\n\t"
                             "s_waitcnt lgkmcnt(0)"
                             : "=&v"(mk[0]), "=&v"(mk[1]), "=&v"(mp[0]), "=&v"(mp[1]), "=&v"(my0[0]), "=&v"(my0[1]),
                               "=&v"(my1[0]), "=&v"(my1[1]), "=&v"(dd[0]), "=&v"(dd[1])
                             : "v"(maddr), "v"(da0), "v"(da1)
                             : "memory");
            } else {
                asm volatile("ds_read_b128 %0, %8\n\t"
                             "ds_read_b128 %1, %8 offset:16\n\t"
                             "ds_read_b128 %2, %8 offset:512\n\t"
                             "ds_read_b128 %3, %8 offset:528\n\t"
                             "ds_read_b128 %4, %8 offset:1024\n\t"
                             "ds_read_b128 %5, %8 offset:1040\n\t"
                             "ds_read2_b64 %6, %9 offset1:64\n\t"
                             "ds_read2_b64 %7, %10 offset1:64\n\t"
                             "s_waitcnt lgkmcnt(0)"
                             : "=&v"(mk[0]), "=&v"(mk[1]), "=&v"(mp[0]), "=&v"(mp[1]), "=&v"(my0[0]), "=&v"(my0[1]),
                               "=&v"(dd[0]), "=&v"(dd[1])
                             : "v"(maddr), "v"(da0), "v"(da1)
                             : "memory");
            }
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int64_t j = 2 * p + e;
                // a row past the block adds zeros to the alpha sums (no branch around
                // them: the accumulators then need no copies across it)
                uint32_t al = 0u;
                double tq[NR];
#pragma unroll
                for (int q = 0; q < NR; ++q) tq[q] = 0.0;
                if (j < nr) {
                    const int h2 = e >> 1, e2 = e & 1;
                    const uint64_t key = ((uint64_t)mk[h2][2 * e2 + 1] << 32) | mk[h2][2 * e2];
                    al = uniform_u32((uint32_t)key);
                    const uint32_t be = uniform_u32((uint32_t)(key >> 32));
                    if (!run || be != cur) {
                        if (run) {
#pragma unroll
                            for (int k = 0; k < NA; ++k) {
                                const double bk = bit_d(cur, k);
#pragma unroll
                                for (int q = 0; q < NR; ++q) wb[q][k] = fma(bk, sb[q], wb[q][k]);
                            }
#pragma unroll
                            for (int q = 0; q < NR; ++q) {
                                bp[q] += sb[q];
                                sb[q] = 0.0;
                            }
                        }
                        cur = be;
                        run = true;
                    }
                    const double ps = u2d(mp[h2], e2);
                    const double d = dd[h2][e2];
                    double c[NR];
#pragma unroll
                    for (int q = 0; q < NR; ++q) {
                        c[q] = fma(-coef, ps, u2d(q == 0 ? my0[h2] : my1[h2], e2));
                        tq[q] = c[q] * d;
                        sb[q] += tq[q];
                    }
#ifdef IRL_VJP_NO_DPP
#pragma unroll
                    for (int k = 0; k < NA; ++k) {
                        const double bk = bit_d(al, k);
#pragma unroll
                        for (int q = 0; q < NR; ++q) wa[q][k] = fma(bk, tq[q], wa[q][k]);
                    }
#endif
                    if (wv == 0) {
                        const uint32_t bits = lane < n ? al : be;
                        const int sh = lane < n ? lane : lane - n;
                        const bool on = lane < V && ((bits >> (sh & 31)) & 1u);
#pragma unroll
                        for (int q = 0; q < NR; ++q) {
                            ax[q] += on ? c[q] : 0.0;
                            a0[q] = fma(c[q], ps, a0[q]);
                        }
                    }
                }
#ifndef IRL_VJP_NO_DPP
                bits_fma<NR, NA>(wa, al, lane, tq);
#endif
            }
            // the pairs' LDS reads have completed (above) before their slots take pairs
            // p + RP and p + RP + 1
            dma_pair(p + RP);
            dma_pair(p + RP + 1);
        }
        // the loads still in flight write LDS only; wait for them before the
        // workgroup ends
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    }
    if (run) {
#pragma unroll
        for (int k = 0; k < NA; ++k) {
            const double bk = bit_d(cur, k);
#pragma unroll
            for (int q = 0; q < NR; ++q) wb[q][k] = fma(bk, sb[q], wb[q][k]);
        }
#pragma unroll
        for (int q = 0; q < NR; ++q) bp[q] += sb[q];
    }
    const int64_t P1 = (int64_t)V * H + H + V + 1;
#pragma unroll
    for (int q = 0; q < NR; ++q) {
        double *out = part + ((int64_t)blockIdx.x * 2 + (NR == 2 ? q : half)) * ldv;
        if (t < H) {
            double *wrow = out + 1 + V + H + (int64_t)t * V;
#pragma unroll
            for (int k = 0; k < NA; ++k)
                if (k < n) {
                    wrow[k] = wa[q][k];
                    wrow[n + k] = wb[q][k];
                }
            out[1 + V + t] = bp[q];
        }
        if (wv == 0) {
            if (lane < V) out[1 + lane] = ax[q];
            if (lane == 0) out[0] = a0[q];
            for (int64_t col = P1 + lane; col < ldv; col += 64) out[col] = 0.0;
        }
    }
}

// ---------------------------------------------------------------------------
// D~ v on selected sets on the vector units, with the occupation sums read from
// tables.  Row r needs t_r[h] = v_b[h] + sum over its occupied orbitals of
// V_W[h][v]; the matrix-core form multiplies the whole 0/1 row of X, half of it
// zeros, on FP64 matrix cores that are no faster than the vector units on this
// part.  Here the alpha and the beta orbitals are each split into groups of 4,
// and for each group and each of its 16 occupation patterns a workgroup tabulates
// the pattern's sum of V_W[h][v] (orbitals in increasing order) for the 64 hidden
// units of a chunk in LDS, so t_r is one table read per group.  A workgroup owns
// a block of rows and walks the hidden chunks in order; each wave owns a
// contiguous part of the block and walks it in 16-row batches (lane l = hidden
// unit 64 c + l, one coalesced 512-byte d segment per row), loads the next
// batch's d, keys and psi while the current one is summed, and forms the 16 row
// sums of d t with one transposed butterfly.  Chunk 0 adds psi_r v_0 and x_r . v_a
// (tables of v_a, read at a uniform address); later chunks add to w in chunk
// order, so the sum is fixed by the launch shape.
#ifndef IRL_LUT_THREADS
#define IRL_LUT_THREADS 1024
#endif
#ifndef IRL_LUT_BLOCKS
#define IRL_LUT_BLOCKS 256
#endif
constexpr int kLutRB = 16;        // rows per batch (one transposed butterfly)
constexpr int kLutThreads = IRL_LUT_THREADS;
constexpr int kLutMaxG = 6;       // groups of 4 orbitals per spin (n <= 24)
constexpr int kLutBlocks = IRL_LUT_BLOCKS;

// row sums of p[0..16) over the wavefront (p is consumed): on return lane l holds
// the sum of row (l >> 2) & 15, the same value in the 4 lanes of a row
__device__ __forceinline__ double rows16_sum(double (&p)[kLutRB], int lane)
{
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const int o = 32 >> s, half = 8 >> s;
        // the choice by bit mask: a select between two elements would become an
        // indexed access and put p in scratch memory
        const uint64_t m = (lane & o) ? ~0ull : 0ull;
#pragma unroll
        for (int k = 0; k < half; ++k) {
            const uint64_t lo = __builtin_bit_cast(uint64_t, p[k]), hi = __builtin_bit_cast(uint64_t, p[k + half]);
            const double send = __builtin_bit_cast(double, (lo & m) | (hi & ~m));
            const double keep = __builtin_bit_cast(double, (hi & m) | (lo & ~m));
            p[k] = keep + __shfl_xor(send, o, kWave);
        }
    }
    double r = p[0];
    r += __shfl_xor(r, 1, kWave);
    r += __shfl_xor(r, 2, kWave);
    return r;
}

// tables of one hidden chunk, shared by the workgroup: spin s (0 alpha, 1 beta),
// group g, pattern p at [s][g][p]
template <int NG>
struct LutShared {
    double lut[2][NG][16][64];   // pattern sums of V_W[64 c + lane][s n + 4 g + j]
    double xlut[2][NG][16];      // pattern sums of v_a[s n + 4 g + j]
};

// the 16 pattern sums of x[0..4) (entries past n are zero), each in increasing
// orbital order: the pattern without its highest bit, plus that bit's entry
__device__ __forceinline__ void pattern_sums(const double (&x)[4], double (&out)[16])
{
    out[0] = 0.0;
#pragma unroll
    for (int p = 1; p < 16; ++p) {
        const int top = p >= 8 ? 3 : p >= 4 ? 2 : p >= 2 ? 1 : 0;
        out[p] = p == (1 << top) ? x[top] : out[p - (1 << top)] + x[top];
    }
}

// one wave's rows [r0, r1) for hidden chunk c (lane = unit 64 c + lane).
// D~ v (FWD false): out = w; FIRST (chunk 0) writes psi v_0 + x . v_a + the chunk's
// sum of d t, later chunks add theirs.  Forward pass (FWD true): t is z = b + W x,
// the chunk's d = 1 - tanh^2 z goes to dout and out = psi gets x . a + the sum of
// tanh z in the same way.
template <int NG, bool FIRST, bool FWD>
__device__ __forceinline__ void lut_rows(const BitsArgs &A, const LutShared<NG> &T, int64_t r0, int64_t r1, int h,
                                         int lane, double bh, double v0, double *__restrict__ out,
                                         double *__restrict__ dout)
{
    const int H = A.H;
    // a lane past H (the last chunk of a width that is not a multiple of 64) reads
    // and writes past every descriptor's end: its d is 0 and its stores are dropped
    const uint32_t dvo = h < H ? (uint32_t)h * 8u : 0x40000000u;
    const int nbatch = (int)((r1 - r0 + kLutRB - 1) / kLutRB);
    uint32_t cur = 0xffffffffu;   // beta string of tb (none yet: strings are < 2^n)
    double tb = 0.0;
    for (int b = 0; b < nbatch; ++b) {
        const int64_t rb = r0 + (int64_t)b * kLutRB;
        const int cnt = r1 - rb < kLutRB ? (int)(r1 - rb) : kLutRB;
        // the batch's d segments, keys and psi through buffer descriptors bounded
        // at its last row (rows past it read as zeros, stores past it are dropped);
        // the 16 rows' loads are in flight together, and the other waves of the
        // SIMD (four per SIMD) keep it busy meanwhile
        const auto rs = __builtin_amdgcn_make_buffer_rsrc((void *)((FWD ? dout : A.dfac) + rb * H), 0,
                                                          cnt * H * 8, kBufWord3);
        double d[kLutRB];
        if (!FWD) {
#pragma unroll
            for (int i = 0; i < kLutRB; ++i)
                d[i] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rs, dvo, i * H * 8, 0));
        }
        const auto rk = __builtin_amdgcn_make_buffer_rsrc((void *)(A.keys + rb), 0, cnt * 8, kBufWord3);
        const uint64_t kl = __builtin_bit_cast(uint64_t, __builtin_amdgcn_raw_buffer_load_b64(rk, lane * 8, 0, 0));
        double pl = 0.0;
        if (FIRST && !FWD) {
            const auto rp = __builtin_amdgcn_make_buffer_rsrc((void *)(A.psi + rb), 0, cnt * 8, kBufWord3);
            pl = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rp, lane * 8, 0, 0));
        }
        // row i's t: bh + its beta part + its alpha part (t0: the first two)
        auto finish = [&](int i, double t) {
            if (FWD) {
                double th, dd;
                tanh_and_d(t, th, dd);
                __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2v, dd), rs, dvo, i * H * 8, 0);
                d[i] = th;
            } else {
                d[i] *= t;
            }
        };
        // one beta string for the whole batch (the usual case: rows ascend
        // beta-major): its part of t is read once; otherwise per row
        const uint32_t khi = (uint32_t)(kl >> 32);
        const uint32_t b0 = (uint32_t)__builtin_amdgcn_readfirstlane((int)khi);
        const bool one_beta = __ballot(lane < cnt && khi != b0) == 0;
        if (one_beta) {
            if (b0 != cur) {
                cur = b0;
                tb = 0.0;
#pragma unroll
                for (int g = 0; g < NG; ++g) tb += T.lut[1][g][(b0 >> (4 * g)) & 15u][lane];
            }
            const double tb0 = bh + tb;
#pragma unroll
            for (int i = 0; i < kLutRB; ++i) {
                const uint32_t oa = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)kl, i);
                double t = tb0;
#pragma unroll
                for (int g = 0; g < NG; ++g) t += T.lut[0][g][(oa >> (4 * g)) & 15u][lane];
                finish(i, t);
            }
        } else {
            cur = 0xffffffffu;
#pragma unroll
            for (int i = 0; i < kLutRB; ++i) {
                const uint32_t occ[2] = {(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)kl, i),
                                         (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(kl >> 32), i)};
                double t = bh;
#pragma unroll
                for (int sp = 0; sp < 2; ++sp)
#pragma unroll
                    for (int g = 0; g < NG; ++g) t += T.lut[sp][g][(occ[sp] >> (4 * g)) & 15u][lane];
                finish(i, t);
            }
        }
        double sum = rows16_sum(d, lane);
        const int j = lane >> 2;
        if (FIRST) {
            // x_j . a (or psi_j v_0 + x_j . v_a) for row j, the (spin, group)
            // tables split over the row's 4 lanes and summed in a fixed order
            const uint64_t kj = __shfl(kl, j, kWave);
            double x = 0.0;
#pragma unroll
            for (int m = 0; m < (2 * NG + 3) / 4; ++m) {
                const int k = 4 * m + (lane & 3);
                const bool beta = k >= NG;
                const int g = beta ? k - NG : k;
                const uint32_t o = beta ? (uint32_t)(kj >> 32) : (uint32_t)kj;
                if (k < 2 * NG) x += T.xlut[beta ? 1 : 0][g][(o >> (4 * g)) & 15u];
            }
            x += __shfl_xor(x, 1, kWave);
            x += __shfl_xor(x, 2, kWave);
            if (FWD)
                sum += x;
            else
                sum += fma(__shfl(pl, j, kWave), v0, x);
        }
        if ((lane & 3) == 0 && j < cnt) {
            const int64_t row = rb + j;
            out[row] = FIRST ? sum : out[row] + sum;
        }
    }
}

// the workgroup's tables for hidden chunk c of M (H x V, row-major) and of the
// visible vector a (xlut, built once by the caller's first call)
template <int NG>
__device__ __forceinline__ void lut_build(LutShared<NG> &T, const double *__restrict__ M, const double *__restrict__ a,
                                          int n, int V, int H, int c, int lane, int wv, int nwv)
{
    if (c == 0 && threadIdx.x < 2 * NG) {
        const int sp = threadIdx.x / NG, g = threadIdx.x % NG;
        double x[4], o[16];
#pragma unroll
        for (int j = 0; j < 4; ++j) x[j] = 4 * g + j < n ? a[sp * n + 4 * g + j] : 0.0;
        pattern_sums(x, o);
#pragma unroll
        for (int p = 0; p < 16; ++p) T.xlut[sp][g][p] = o[p];
    }
    // pattern sums of M for unit h: wave wv takes (spin, group) pairs wv, wv + nwv, ...
    const int h = 64 * c + lane;
    for (int q = wv; q < 2 * NG; q += nwv) {
        const int sp = q / NG, g = q % NG;
        double x[4], o[16];
#pragma unroll
        for (int j = 0; j < 4; ++j) x[j] = (h < H && 4 * g + j < n) ? M[(size_t)h * V + sp * n + 4 * g + j] : 0.0;
        pattern_sums(x, o);
#pragma unroll
        for (int p = 0; p < 16; ++p) T.lut[sp][g][p][lane] = o[p];
    }
}

// this wave's part of the workgroup's block of rows: whole batches, in wave order.
// Blocks hold a multiple of kLutRB rows, so every batch starts at a multiple of
// kLutRB and a row's place in the butterfly (row mod kLutRB) does not depend on the
// workgroup count: the sums are the same for any grid.
__device__ __forceinline__ void lut_wave_rows(int64_t ns, int wv, int nwv, int64_t &r0, int64_t &r1)
{
    const int64_t bper = ((ns + gridDim.x - 1) / gridDim.x + kLutRB - 1) / kLutRB * kLutRB;
    r0 = (int64_t)blockIdx.x * bper;
    r1 = r0 + bper < ns ? r0 + bper : ns;
    if (r0 > ns) r0 = ns;
    const int64_t nb = (r1 - r0 + kLutRB - 1) / kLutRB, per = (nb + nwv - 1) / nwv;
    const int64_t q0 = r0 + (int64_t)wv * per * kLutRB, q1 = q0 + per * kLutRB;
    r1 = q1 < r1 ? q1 : r1;
    r0 = q0 < r1 ? q0 : r1;
}

template <int NG>
__global__ __launch_bounds__(kLutThreads) void k_fac_jvp_lut(BitsArgs A, const double *__restrict__ v, int zero_v0,
                                                             double *__restrict__ w)
{
    static_assert(NG >= 1 && NG <= kLutMaxG, "orbital groups");
    __shared__ LutShared<NG> T;
    const int lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    constexpr int nwv = kLutThreads / 64;
    const int V = A.V, H = A.H;
    int64_t r0, r1;
    lut_wave_rows(A.ns, wv, nwv, r0, r1);
    const double *va = v + 1, *vb = v + 1 + V, *vW = v + 1 + V + H;
    const double v0 = zero_v0 ? 0.0 : v[0];
    for (int c = 0; 64 * c < H; ++c) {
        __syncthreads();   // the previous chunk's tables are no longer read
        lut_build(T, vW, va, A.n, V, H, c, lane, wv, nwv);
        __syncthreads();
        const int h = 64 * c + lane;
        const double bh = h < H ? vb[h] : 0.0;
        if (c == 0)
            lut_rows<NG, true, false>(A, T, r0, r1, h, lane, bh, v0, w, nullptr);
        else
            lut_rows<NG, false, false>(A, T, r0, r1, h, lane, bh, v0, w, nullptr);
    }
}

// forward pass on selected sets with the same tables (of W and a): psi and d
template <int NG>
__global__ __launch_bounds__(kLutThreads) void k_fac_forward_lut(BitsArgs A, const double *__restrict__ theta,
                                                                 double *__restrict__ psi, double *__restrict__ dfac)
{
    static_assert(NG >= 1 && NG <= kLutMaxG, "orbital groups");
    __shared__ LutShared<NG> T;
    const int lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    constexpr int nwv = kLutThreads / 64;
    const int V = A.V, H = A.H;
    int64_t r0, r1;
    lut_wave_rows(A.ns, wv, nwv, r0, r1);
    const double *a = theta, *bb = theta + V, *W = theta + V + H;
    for (int c = 0; 64 * c < H; ++c) {
        __syncthreads();
        lut_build(T, W, a, A.n, V, H, c, lane, wv, nwv);
        __syncthreads();
        const int h = 64 * c + lane;
        const double bh = h < H ? bb[h] : 0.0;
        if (c == 0)
            lut_rows<NG, true, true>(A, T, r0, r1, h, lane, bh, 0.0, psi, dfac);
        else
            lut_rows<NG, false, true>(A, T, r0, r1, h, lane, bh, 0.0, psi, dfac);
    }
}

// the vector-unit forms apply to these rows: not the full-space kernels, n <= 24,
// 48 <= H <= 256
bool fac_bits_ok(const irl_system *s, int H)
{
#ifdef IRL_FAC_NO_BITS
    return false;
#endif
    return s->n <= kBitsMaxN && H >= kBitsMinH && H <= kBitsMaxH;
}

// the table-driven forward pass and D~ v apply to these rows: not the full-space
// kernels, n <= 24, H >= 48 (a last chunk of a width that is not a multiple of 64
// leaves its lanes past H idle; narrower networks keep the matrix-core forms)
bool fac_lut_ok(const irl_system *s, int H)
{
#ifdef IRL_FAC_NO_LUT
    return false;
#endif
    return s->n <= kBitsMaxN && H >= kBitsMinH;
}

// row blocks of the table-driven kernels: at most kLutBlocks (or the system's
// tuned count), at least 128 rows each.  Each row's sums are formed by one wave in
// a fixed order, so the count moves rows between workgroups and nothing else.
unsigned lut_blocks(const irl_system *s, int64_t ns)
{
    const int64_t cap = s->tune_lut_blocks > 0 ? s->tune_lut_blocks : kLutBlocks;
    int64_t per = (ns + cap - 1) / cap;
    if (per < 128) per = 128;
    return (unsigned)((ns + per - 1) / per);
}

int fac_bits_blocks(int64_t ns)
{
    int64_t per = (ns + kBitsBlocks - 1) / kBitsBlocks;
    if (per < 64) per = 64;
    const int64_t nb = (ns + per - 1) / per;
    return (int)(nb < 1 ? 1 : nb);
}

template <int NA>
static void launch_bits_na(const BitsArgs &B, int nblk, const double *y0, const double *y1, const double *coefp,
                           double *part, int64_t ldv, int half, hipStream_t st)
{
    const unsigned threads = (unsigned)(64 * ((B.H + 63) / 64));
#ifndef IRL_FAC_NO_RING
    if (B.H % 64 == 0) {
        if (y1)
            k_fac_vjp_ring<2, NA><<<nblk, threads, 0, st>>>(B, y0, y1, coefp, part, ldv, nblk, 0);
        else
            k_fac_vjp_ring<1, NA><<<nblk, threads, 0, st>>>(B, y0, nullptr, coefp, part, ldv, nblk, half);
        return;
    }
#endif
    if (y1)
        k_fac_vjp_bits<2, NA><<<nblk, threads, 0, st>>>(B, y0, y1, coefp, part, ldv, nblk, 0);
    else
        k_fac_vjp_bits<1, NA><<<nblk, threads, 0, st>>>(B, y0, nullptr, coefp, part, ldv, nblk, half);
}

// D~^T [y0, y1] (y1 == nullptr: D~^T y0 into half `half`) on the vector units
static hipError_t launch_vjp_bits(const irl_system *s, const BitsArgs &B, int nblk, const double *y0,
                                  const double *y1, const double *coefp, double *part, int64_t ldv, int half,
                                  hipStream_t st)
{
    switch ((s->n + 3) / 4) {
    case 0: case 1: case 2: launch_bits_na<8>(B, nblk, y0, y1, coefp, part, ldv, half, st); break;
    case 3: launch_bits_na<12>(B, nblk, y0, y1, coefp, part, ldv, half, st); break;
    case 4: launch_bits_na<16>(B, nblk, y0, y1, coefp, part, ldv, half, st); break;
    case 5: launch_bits_na<20>(B, nblk, y0, y1, coefp, part, ldv, half, st); break;
    default: launch_bits_na<24>(B, nblk, y0, y1, coefp, part, ldv, half, st); break;
    }
    return hipGetLastError();
}

bool fac_shape_ok(const irl_system *s, const WsLayout &L)
{
    const int V = 2 * s->n;
    return (L.flags & IRL_WS_FACTORED) && L.hfac >= 1 && V >= 1 && V <= 64 &&
           (int64_t)V * L.hfac + L.hfac + V + 1 <= L.ldv;
}

// the string-split backward product applies to these rows of this workspace
bool fac_full_ok(const irl_system *s, const WsLayout &L, const FacRows &R)
{
    return L.kf_S > 0 && s->full && R.keys == s->d.keys && R.ns == s->ns && s->nA * s->nB == s->ns &&
           s->d.strA && s->d.strB && L.hfac >= 1;
}

FullArgs full_args(const irl_system *s, const WsLayout &L, const FacRows &R, const double *y0, const double *y1,
                   const double *coefp, int half, double *part)
{
    const int S = L.kf_S;
    FullArgs F;
    F.dfac = R.dfac;
    F.psi = R.psi;
    F.y0 = y0;
    F.y1 = y1;
    F.coefp = coefp;
    F.strA = s->d.strA;
    F.strB = s->d.strB;
    F.nA = s->nA;
    F.nB = s->nB;
    F.aper = (s->nA + S - 1) / S;
    F.ldv = L.ldv;
    F.n = s->n;
    F.H = L.hfac;
    F.V = 2 * s->n;
    F.S = S;
    F.half = half;
    F.part = part;
    return F;
}

template <int NA>
hipError_t vjp_full_na(const irl_system *s, const WsLayout &L, void *ws, const FacRows &R, const double *y0,
                       const double *y1, const double *coefp, int half, int nblk, hipStream_t st)
{
    const int H = L.hfac, S = L.kf_S;
    const int64_t nbt = (s->nB + kFullTB - 1) / kFullTB;
    if (nblk != nbt * S) return hipErrorInvalidValue;
    const FullArgs F = full_args(s, L, R, y0, y1, coefp, half, ws_ptr<double>(ws, L.off_part));
    const dim3 grid((unsigned)((H + 63) / 64), (unsigned)nblk);
    if (y1)
        k_fac_vjp_full<2, NA, kFullPD><<<grid, 256, 0, st>>>(F);
    else
        k_fac_vjp_full<1, NA, kFullPD><<<grid, 256, 0, st>>>(F);
    return hipGetLastError();
}

}  // namespace

int fac_full_ranges(int64_t nA, int64_t nB, int n, int H)
{
    // one partial row per workgroup: at most kStreamBlocks of them, at least 16
    // alpha strings (4 per wave) per range
    const int64_t nbt = (nB + kFullTB - 1) / kFullTB;
    if (nA < 1 || nB < 1 || nA * nB < kFullMinRows || n < 1 || n > kFullMaxN || H < 1 || nbt > kStreamBlocks)
        return 0;
    int64_t S = kStreamBlocks / nbt;
    const int64_t smax = (nA + 15) / 16;
    if (S > smax) S = smax;
    return (int)(S < 1 ? 1 : S);
}

int fac_jvp_uses_lut(const irl_system *s, int64_t ns, int H)
{
    const bool full = s->full && ns == s->ns && s->nA * s->nB == s->ns && s->d.strA && s->d.strB &&
                      fac_full_ranges(s->nA, s->nB, s->n, H) > 0;
    return (!(full && H <= 64) && fac_lut_ok(s, H)) ? 1 : 0;
}

int fac_vjp_blocks(const irl_system *s, const WsLayout &L)
{
    if (L.kf_S > 0 && s->full) return (int)(((s->nB + kFullTB - 1) / kFullTB) * L.kf_S);
    return fac_row_blocks(s, L);
}

FacRows fac_rows(const irl_system *s, const WsLayout &L, void *ws)
{
    return FacRows{s->d.keys, L.ns, ws_ptr<double>(ws, L.off_psi), ws_ptr<double>(ws, L.off_fac)};
}

hipError_t launch_fac_forward(const irl_system *s, const WsLayout &L, void *ws, const double *theta,
                              hipStream_t st)
{
    if (!fac_shape_ok(s, L)) return hipErrorInvalidValue;
    const int V = 2 * s->n, H = L.hfac;
    double *psi = ws_ptr<double>(ws, L.off_psi), *dfac = ws_ptr<double>(ws, L.off_fac);
    const FacRows R = fac_rows(s, L, ws);
    if (fac_full_ok(s, L, R) && H <= 64) {
        const FullArgs F = full_args(s, L, R, nullptr, nullptr, nullptr, 0, nullptr);
        const unsigned grid = (unsigned)(((s->nB + kFullTB - 1) / kFullTB) * L.kf_S);
        switch ((s->n + 3) / 4) {
        case 1: k_fac_forward_full<4><<<grid, 256, 0, st>>>(F, theta, psi, dfac); break;
        case 2: k_fac_forward_full<8><<<grid, 256, 0, st>>>(F, theta, psi, dfac); break;
        case 3: k_fac_forward_full<12><<<grid, 256, 0, st>>>(F, theta, psi, dfac); break;
        default: k_fac_forward_full<16><<<grid, 256, 0, st>>>(F, theta, psi, dfac); break;
        }
        return hipGetLastError();
    }
#ifndef IRL_FAC_NO_LUT_FWD
    if (fac_lut_ok(s, H)) {
        const BitsArgs B{R.keys, R.psi, R.dfac, R.ns, s->n, V, H};
        const unsigned nblk = lut_blocks(s, R.ns);
        switch ((s->n + 3) / 4) {
        case 1: k_fac_forward_lut<1><<<nblk, kLutThreads, 0, st>>>(B, theta, psi, dfac); break;
        case 2: k_fac_forward_lut<2><<<nblk, kLutThreads, 0, st>>>(B, theta, psi, dfac); break;
        case 3: k_fac_forward_lut<3><<<nblk, kLutThreads, 0, st>>>(B, theta, psi, dfac); break;
        case 4: k_fac_forward_lut<4><<<nblk, kLutThreads, 0, st>>>(B, theta, psi, dfac); break;
        case 5: k_fac_forward_lut<5><<<nblk, kLutThreads, 0, st>>>(B, theta, psi, dfac); break;
        default: k_fac_forward_lut<6><<<nblk, kLutThreads, 0, st>>>(B, theta, psi, dfac); break;
        }
        return hipGetLastError();
    }
#endif
    switch ((V + 7) / 8) {
    case 1: forward_ks<2>(s, L, V, H, theta, psi, dfac, st); break;
    case 2: forward_ks<4>(s, L, V, H, theta, psi, dfac, st); break;
    case 3: forward_ks<6>(s, L, V, H, theta, psi, dfac, st); break;
    case 4: forward_ks<8>(s, L, V, H, theta, psi, dfac, st); break;
    case 5: forward_ks<10>(s, L, V, H, theta, psi, dfac, st); break;
    case 6: forward_ks<12>(s, L, V, H, theta, psi, dfac, st); break;
    case 7: forward_ks<14>(s, L, V, H, theta, psi, dfac, st); break;
    default: forward_ks<16>(s, L, V, H, theta, psi, dfac, st); break;
    }
    return hipGetLastError();
}


hipError_t launch_fac_jvp_rows(const irl_system *s, const WsLayout &L, const FacRows &R, const double *v,
                               int zero_v0, double *w, hipStream_t st)
{
    if (!fac_shape_ok(s, L) || R.ns < 1) return hipErrorInvalidValue;
    const int V = 2 * s->n, H = L.hfac;
    if (fac_full_ok(s, L, R) && H <= 64) {
        FullArgs F = full_args(s, L, R, nullptr, nullptr, nullptr, 0, nullptr);
        const unsigned grid = (unsigned)(((s->nB + kFullTB - 1) / kFullTB) * L.kf_S);
        switch ((s->n + 3) / 4) {
        case 1: k_fac_jvp_full<4><<<grid, 256, 0, st>>>(F, v, zero_v0, w); break;
        case 2: k_fac_jvp_full<8><<<grid, 256, 0, st>>>(F, v, zero_v0, w); break;
        case 3: k_fac_jvp_full<12><<<grid, 256, 0, st>>>(F, v, zero_v0, w); break;
        default: k_fac_jvp_full<16><<<grid, 256, 0, st>>>(F, v, zero_v0, w); break;
        }
        return hipGetLastError();
    }
    if (fac_lut_ok(s, H)) {
        const BitsArgs B{R.keys, R.psi, R.dfac, R.ns, s->n, V, H};
        const unsigned nblk = lut_blocks(s, R.ns);
        switch ((s->n + 3) / 4) {
        case 1: k_fac_jvp_lut<1><<<nblk, kLutThreads, 0, st>>>(B, v, zero_v0, w); break;
        case 2: k_fac_jvp_lut<2><<<nblk, kLutThreads, 0, st>>>(B, v, zero_v0, w); break;
        case 3: k_fac_jvp_lut<3><<<nblk, kLutThreads, 0, st>>>(B, v, zero_v0, w); break;
        case 4: k_fac_jvp_lut<4><<<nblk, kLutThreads, 0, st>>>(B, v, zero_v0, w); break;
        case 5: k_fac_jvp_lut<5><<<nblk, kLutThreads, 0, st>>>(B, v, zero_v0, w); break;
        default: k_fac_jvp_lut<6><<<nblk, kLutThreads, 0, st>>>(B, v, zero_v0, w); break;
        }
        return hipGetLastError();
    }
    switch ((V + 7) / 8) {
    case 1: jvp_ks<2>(s, R, V, H, v, zero_v0, w, st); break;
    case 2: jvp_ks<4>(s, R, V, H, v, zero_v0, w, st); break;
    case 3: jvp_ks<6>(s, R, V, H, v, zero_v0, w, st); break;
    case 4: jvp_ks<8>(s, R, V, H, v, zero_v0, w, st); break;
    case 5: jvp_ks<10>(s, R, V, H, v, zero_v0, w, st); break;
    case 6: jvp_ks<12>(s, R, V, H, v, zero_v0, w, st); break;
    case 7: jvp_ks<14>(s, R, V, H, v, zero_v0, w, st); break;
    default: jvp_ks<16>(s, R, V, H, v, zero_v0, w, st); break;
    }
    return hipGetLastError();
}

hipError_t launch_fac_jvp(const irl_system *s, const WsLayout &L, void *ws, const double *v, int zero_v0,
                          double *w, hipStream_t st)
{
    return launch_fac_jvp_rows(s, L, fac_rows(s, L, ws), v, zero_v0, w, st);
}

// row blocks of the backward pass: at H = 64 the 256 row blocks x 2 hidden-unit
// groups are 2048 waves, one round on the chip at two waves per SIMD (512 row
// blocks took 0.229 against 0.221 ms per c2 pass, with twice the partial rows)
constexpr int kFacRowBlocks = 256;

int fac_row_blocks_n(const irl_system *s, int64_t ns, int hfac)
{
    if (fac_bits_ok(s, hfac)) return fac_bits_blocks(ns);
    const int htiles = (hfac + 63) / 64;
    int nblk = kFacRowBlocks / (htiles > 0 ? htiles : 1);
    if (nblk < 1) nblk = 1;
    if (nblk > (ns + 15) / 16) nblk = (int)((ns + 15) / 16);
    return nblk < 1 ? 1 : nblk;
}

int fac_row_blocks(const irl_system *s, const WsLayout &L)
{
    return fac_row_blocks_n(s, L.ns, L.hfac);
}

hipError_t launch_fac_vjp_rows(const irl_system *s, const WsLayout &L, void *ws, const FacRows &R,
                               const double *y0, const double *y1, const double *coefp, int half, int nblk,
                               hipStream_t st)
{
    if (!fac_shape_ok(s, L) || R.ns < 1 || nblk < 1 || nblk > kStreamBlocks || !y0) return hipErrorInvalidValue;
    if (fac_full_ok(s, L, R)) {
        switch ((s->n + 3) / 4) {
        case 1: return vjp_full_na<4>(s, L, ws, R, y0, y1, coefp, half, nblk, st);
        case 2: return vjp_full_na<8>(s, L, ws, R, y0, y1, coefp, half, nblk, st);
        case 3: return vjp_full_na<12>(s, L, ws, R, y0, y1, coefp, half, nblk, st);
        default: return vjp_full_na<16>(s, L, ws, R, y0, y1, coefp, half, nblk, st);
        }
    }
    const int V = 2 * s->n, H = L.hfac;
    double *part = ws_ptr<double>(ws, L.off_part);
    if (fac_bits_ok(s, H)) {
        const BitsArgs B{R.keys, R.psi, R.dfac, R.ns, s->n, V, H};
        return launch_vjp_bits(s, B, nblk, y0, y1, coefp, part, L.ldv, half, st);
    }
    const int nt = (V + 15) / 16;
    if (y1) {
        switch (nt) {
        case 1: vjp_nt<1, 2>(s, L, R, V, H, y0, y1, coefp, part, nblk, 0, st); break;
        case 2: vjp_nt<2, 2>(s, L, R, V, H, y0, y1, coefp, part, nblk, 0, st); break;
        case 3: vjp_nt<3, 2>(s, L, R, V, H, y0, y1, coefp, part, nblk, 0, st); break;
        default: vjp_nt<4, 2>(s, L, R, V, H, y0, y1, coefp, part, nblk, 0, st); break;
        }
    } else {
        switch (nt) {
        case 1: vjp_nt<1, 1>(s, L, R, V, H, y0, nullptr, coefp, part, nblk, half, st); break;
        case 2: vjp_nt<2, 1>(s, L, R, V, H, y0, nullptr, coefp, part, nblk, half, st); break;
        case 3: vjp_nt<3, 1>(s, L, R, V, H, y0, nullptr, coefp, part, nblk, half, st); break;
        default: vjp_nt<4, 1>(s, L, R, V, H, y0, nullptr, coefp, part, nblk, half, st); break;
        }
    }
    return hipGetLastError();
}

hipError_t launch_fac_vjp(const irl_system *s, const WsLayout &L, void *ws, const double *y0, const double *y1,
                          const double *coefp, int half, int nblk, hipStream_t st)
{
    return launch_fac_vjp_rows(s, L, ws, fac_rows(s, L, ws), y0, y1, coefp, half, nblk, st);
}

}  // namespace irl
