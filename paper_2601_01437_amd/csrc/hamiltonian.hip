// u = H w restricted to the determinant set (Slater-Condon rules) on gfx950.
//
// Hamiltonian of Methods, "Wave Function Ansatz":
//   H = sum h_pq a+_p a_q + 1/2 sum (pq|rs) a+_p a+_r a_s a_q  (spin-orbitals,
//   chemists' integrals, alpha spin-orbitals before beta ones).
// A determinant is a+_{k1} a+_{k2} ... |0> with ascending spin-orbitals; moving
// an electron i -> a inside one spin string gives the sign
// (-1)^popcount(occupied bits strictly between i and a).  Elements:
//   single i->a (spin s):  h_ia + sum_{j in s}[(ia|jj) - (ij|ja)] + sum_{j in s'} (ia|jj)
//   same-spin double i<j -> a<b (i->a, then j->b, signs multiplied):
//                          (ia|jb) - (ib|ja)
//   opposite-spin double alpha i->a, beta j->b:  (ia|jb)
// Targets outside the set are dropped (Hamiltonian projected onto the set).
//
// Kernel: the general "pull" form, one 64-lane wavefront per determinant.  The
// lanes first build the row's single-excitation and orbital-pair lists in
// LDS, then stride over all singles and doubles, look the target up (string
// ranks for a full space, an open-addressing hash otherwise), gather w and
// accumulate; a fixed shuffle tree reduces the lanes, so results are bitwise
// reproducible.
#include "internal.h"

namespace irl {

struct HamArgs {
    int n, na, nb;
    int64_t ns, nA;
    const uint64_t *keys;
    const double *diag, *h, *g;
    const uint64_t *hkeys;
    const int32_t *hrows;
    uint64_t hmask;
    const int32_t *rankA, *rankB;
};

__device__ __forceinline__ uint64_t mix64h(uint64_t x)
{
    x ^= x >> 33;
    x *= 0xff51afd7ed558ccdull;
    x ^= x >> 33;
    x *= 0xc4ceb9fe1a85ec53ull;
    x ^= x >> 33;
    return x;
}

__device__ __forceinline__ double gint(const double *g, int n, int p, int q, int r, int s)
{
    return g[(((size_t)p * n + q) * n + r) * n + s];
}

// (-1)^popcount(bits strictly between i and a), i != a
__device__ __forceinline__ int move_sign(uint32_t bits, int i, int a)
{
    int lo = min(i, a), hi = max(i, a);
    uint32_t mask = ((1u << hi) - 1u) & ~((2u << lo) - 1u);
    return (__popc(bits & mask) & 1) ? -1 : 1;
}

__device__ __forceinline__ double single_value(const double *h, const double *g, int n,
                                               uint32_t same, uint32_t other, int i, int a)
{
    double v = h[i * n + a];
    for (uint32_t b = same; b; b &= b - 1) {
        int j = __ffs(b) - 1;
        v += gint(g, n, i, a, j, j) - gint(g, n, i, j, j, a);
    }
    for (uint32_t b = other; b; b &= b - 1) {
        int j = __ffs(b) - 1;
        v += gint(g, n, i, a, j, j);
    }
    return v;
}

template <bool FULL>
__device__ __forceinline__ int64_t find_row(const HamArgs &A, uint32_t al, uint32_t be)
{
    if (FULL) {
        return (int64_t)A.rankB[be] * A.nA + A.rankA[al];
    } else {
        uint64_t key = (uint64_t)al | ((uint64_t)be << 32);
        uint64_t slot = mix64h(key) & A.hmask;
        for (uint64_t probe = 0; probe <= A.hmask; ++probe) {
            uint64_t k = A.hkeys[slot];
            if (k == key) return A.hrows[slot];
            if (k == kEmptyKey) return -1;
            slot = (slot + 1) & A.hmask;
        }
        return -1;
    }
}

constexpr int kMaxSingles = 256;   // n <= 32: na * (n - na) <= 256
constexpr int kMaxPairs = 496;     // C(32, 2)

struct WaveLists {
    uint32_t sA[kMaxSingles];      // i | a << 5 | (sign < 0) << 10
    uint32_t sAstr[kMaxSingles];
    uint32_t sB[kMaxSingles];
    uint32_t sBstr[kMaxSingles];
    uint16_t poA[kMaxPairs], pvA[kMaxPairs], poB[kMaxPairs], pvB[kMaxPairs];  // i | j << 8
};

// k-th set bit (0-based) of x
__device__ __forceinline__ int nth_bit(uint32_t x, int k)
{
    for (int t = 0; t < k; ++t) x &= x - 1;
    return __ffs(x) - 1;
}

// lists of single moves and orbital pairs of one spin string, built by the 64 lanes
__device__ void build_lists(uint32_t bits, int n, int ne, uint32_t *s, uint32_t *sstr, uint16_t *po,
                            uint16_t *pv, int lane)
{
    const int nv = n - ne;
    const uint32_t full = (n == 32) ? 0xffffffffu : ((1u << n) - 1u);
    const uint32_t vir = ~bits & full;
    for (int e = lane; e < ne * nv; e += kWave) {
        int x = e / nv, y = e - x * nv;
        int i = nth_bit(bits, x), a = nth_bit(vir, y);
        int sg = move_sign(bits, i, a);
        s[e] = (uint32_t)i | ((uint32_t)a << 5) | ((sg < 0 ? 1u : 0u) << 10);
        sstr[e] = (bits & ~(1u << i)) | (1u << a);
    }
    // ordered pairs x < y of occupied and of virtual orbitals
    for (int t = lane; t < ne * ne; t += kWave) {
        int x = t / ne, y = t - x * ne;
        if (x < y) {
            int pos = x * ne - x * (x + 1) / 2 + (y - x - 1);
            po[pos] = (uint16_t)(nth_bit(bits, x) | (nth_bit(bits, y) << 8));
        }
    }
    for (int t = lane; t < nv * nv; t += kWave) {
        int x = t / nv, y = t - x * nv;
        if (x < y) {
            int pos = x * nv - x * (x + 1) / 2 + (y - x - 1);
            pv[pos] = (uint16_t)(nth_bit(vir, x) | (nth_bit(vir, y) << 8));
        }
    }
}

__device__ __forceinline__ double wave_sum(double v)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

// Evaluate the candidates of one determinant on one lane (stride 64).  OP is
// called with (target row, sign, kind, value) for every target inside the set.
template <bool FULL, typename OP>
__device__ __forceinline__ void visit_row(const HamArgs &A, const WaveLists &L, uint32_t al,
                                          uint32_t be, int lane, int stride, OP op)
{
    const int n = A.n, na = A.na, nb = A.nb, va = n - na, vb = n - nb;
    // alpha and beta singles
    for (int spin = 0; spin < 2; ++spin) {
        const int cnt = spin ? nb * vb : na * va;
        const uint32_t *s = spin ? L.sB : L.sA;
        const uint32_t *ss = spin ? L.sBstr : L.sAstr;
        uint32_t same = spin ? be : al, other = spin ? al : be;
        for (int e = lane; e < cnt; e += stride) {
            uint32_t p = s[e];
            int i = p & 31, a = (p >> 5) & 31, sg = (p >> 10) & 1 ? -1 : 1;
            int64_t r = spin ? find_row<FULL>(A, al, ss[e]) : find_row<FULL>(A, ss[e], be);
            if (r >= 0) op(r, sg, spin ? 2 : 1, sg * single_value(A.h, A.g, n, same, other, i, a));
        }
    }
    // same-spin doubles
    for (int spin = 0; spin < 2; ++spin) {
        const int ne = spin ? nb : na, nv = spin ? vb : va;
        const int npo = ne * (ne - 1) / 2, npv = nv * (nv - 1) / 2;
        const int cnt = npo * npv;
        if (cnt == 0) continue;
        const uint16_t *po = spin ? L.poB : L.poA, *pv = spin ? L.pvB : L.pvA;
        uint32_t bits = spin ? be : al;
        int xo = lane / npv, xv = lane - xo * npv;
        const int step_o = stride / npv, step_v = stride - step_o * npv;
        for (int e = lane; e < cnt; e += stride) {
            int i = po[xo] & 255, j = po[xo] >> 8, a = pv[xv] & 255, b = pv[xv] >> 8;
            int s1 = move_sign(bits, i, a);
            uint32_t b1 = (bits & ~(1u << i)) | (1u << a);
            int s2 = move_sign(b1, j, b);
            uint32_t b2 = (b1 & ~(1u << j)) | (1u << b);
            int64_t r = spin ? find_row<FULL>(A, al, b2) : find_row<FULL>(A, b2, be);
            if (r >= 0) {
                double v = gint(A.g, n, i, a, j, b) - gint(A.g, n, i, b, j, a);
                op(r, s1 * s2, spin ? 4 : 3, (s1 * s2) * v);
            }
            xv += step_v;
            xo += step_o;
            if (xv >= npv) { xv -= npv; ++xo; }
        }
    }
    // opposite-spin doubles
    {
        const int cA = na * va, cB = nb * vb, cnt = cA * cB;
        if (cnt > 0) {
            int xa = lane / cB, xb = lane - xa * cB;
            const int step_a = stride / cB, step_b = stride - step_a * cB;
            for (int e = lane; e < cnt; e += stride) {
                uint32_t pa = L.sA[xa], pb = L.sB[xb];
                int i = pa & 31, a = (pa >> 5) & 31, j = pb & 31, b = (pb >> 5) & 31;
                int sg = (((pa >> 10) ^ (pb >> 10)) & 1) ? -1 : 1;
                int64_t r = find_row<FULL>(A, L.sAstr[xa], L.sBstr[xb]);
                if (r >= 0) op(r, sg, 5, sg * gint(A.g, n, i, a, j, b));
                xb += step_b;
                xa += step_a;
                if (xb >= cB) { xb -= cB; ++xa; }
            }
        }
    }
}

template <bool FULL>
__global__ __launch_bounds__(256) void k_ham_pull(HamArgs A, const double *__restrict__ w,
                                                  double *__restrict__ u)
{
    __shared__ WaveLists lists[4];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    WaveLists &L = lists[wv];
    const int64_t nwaves = (int64_t)gridDim.x * 4;
    for (int64_t row = (int64_t)blockIdx.x * 4 + wv; row < A.ns; row += nwaves) {
        uint64_t key = A.keys[row];
        uint32_t al = (uint32_t)key, be = (uint32_t)(key >> 32);
        build_lists(al, A.n, A.na, L.sA, L.sAstr, L.poA, L.pvA, lane);
        build_lists(be, A.n, A.nb, L.sB, L.sBstr, L.poB, L.pvB, lane);
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        double acc = 0.0;
        visit_row<FULL>(A, L, al, be, lane, kWave,
                        [&](int64_t r, int, int, double v) { acc += v * w[r]; });
        acc = wave_sum(acc);
        if (lane == 0) u[row] = A.diag[row] * w[row] + acc;
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
}

static HamArgs ham_args(const irl_system *s)
{
    HamArgs A;
    A.n = s->n;
    A.na = s->na;
    A.nb = s->nb;
    A.ns = s->ns;
    A.nA = s->nA;
    A.keys = s->d.keys;
    A.diag = s->d.diag;
    A.h = s->d.h;
    A.g = s->d.g;
    A.hkeys = s->d.hkeys;
    A.hrows = s->d.hrows;
    A.hmask = s->d.hcap ? s->d.hcap - 1 : 0;
    A.rankA = s->d.rankA;
    A.rankB = s->d.rankB;
    return A;
}

hipError_t launch_ham_apply(const irl_system *s, const double *w, double *u, hipStream_t st)
{
    HamArgs A = ham_args(s);
    int64_t blocks = (s->ns + 3) / 4;
    if (blocks > 65536) blocks = 65536;
    if (s->full && s->ham_kernel == 0 && s->d.hkeys == nullptr)
        k_ham_pull<true><<<(unsigned)blocks, 256, 0, st>>>(A, w, u);
    else if (s->d.hkeys != nullptr)
        k_ham_pull<false><<<(unsigned)blocks, 256, 0, st>>>(A, w, u);
    else
        k_ham_pull<true><<<(unsigned)blocks, 256, 0, st>>>(A, w, u);
    return hipGetLastError();
}

// Connections of one row (debug surface): same candidate enumeration as the
// apply kernel, one lane, written in enumeration order.
template <bool FULL>
__global__ void k_ham_row_list(HamArgs A, int64_t row, int32_t *tgt, int8_t *sign, uint8_t *kind,
                               double *val, int32_t *count, int cap)
{
    __shared__ WaveLists L;
    const int lane = threadIdx.x;
    uint64_t key = A.keys[row];
    uint32_t al = (uint32_t)key, be = (uint32_t)(key >> 32);
    build_lists(al, A.n, A.na, L.sA, L.sAstr, L.poA, L.pvA, lane);
    build_lists(be, A.n, A.nb, L.sB, L.sBstr, L.poB, L.pvB, lane);
    __syncthreads();
    if (lane != 0) return;
    int c = 0;
    visit_row<FULL>(A, L, al, be, 0, 1, [&](int64_t r, int sg, int k, double v) {
        if (c < cap) {
            tgt[c] = (int32_t)r;
            sign[c] = (int8_t)sg;
            kind[c] = (uint8_t)k;
            val[c] = v;
        }
        ++c;
    });
    *count = c;
}

hipError_t launch_ham_row_list(const irl_system *s, int64_t row, int32_t *tgt, int8_t *sign,
                               uint8_t *kind, double *val, int32_t *count, int cap,
                               hipStream_t st)
{
    HamArgs A = ham_args(s);
    if (s->d.hkeys != nullptr)
        k_ham_row_list<false><<<1, 64, 0, st>>>(A, row, tgt, sign, kind, val, count, cap);
    else
        k_ham_row_list<true><<<1, 64, 0, st>>>(A, row, tgt, sign, kind, val, count, cap);
    return hipGetLastError();
}

hipError_t launch_product_tables(irl_system *, hipStream_t) { return hipSuccess; }

}  // namespace irl
