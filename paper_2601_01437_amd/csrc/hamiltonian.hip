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

typedef HamView HamArgs;

__device__ __forceinline__ uint64_t mix64h(uint64_t x)
{
    x ^= x >> 33;
    x *= 0xff51afd7ed558ccdull;
    x ^= x >> 33;
    x *= 0xc4ceb9fe1a85ec53ull;
    x ^= x >> 33;
    return x;
}

// (pq|rs) of the n^4 chemists' integrals; n <= 32, so the index fits in 32 bits
// (24-bit multiply-adds instead of a 64-bit multiply chain per integral)
__device__ __forceinline__ double gint(const double *g, int n, int p, int q, int r, int s)
{
    const uint32_t un = (uint32_t)n;
    return g[((((uint32_t)p * un + (uint32_t)q) * un + (uint32_t)r) * un + (uint32_t)s)];
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

// key -> row lookup of the per-determinant kernels (LookupMode):
//   kLkRanks   full space: rank(beta) * nA + rank(alpha)
//   kLkHash    any set: membership bitmap, then open-addressing hash
//   kLkBlocks  selected set: beta -> contiguous row block, binary search on alpha

// row of alpha string `al` inside the rows [lo, hi) that share one beta string: a
// search of fixed length (ceil(log2(hi - lo)) halvings, the same for every lane that
// searches the same block) over the keys' low words, then one equality test
__device__ __forceinline__ int64_t search_block(const uint64_t *keys, int64_t lo, int64_t hi,
                                                uint32_t al)
{
    const uint32_t *alpha = reinterpret_cast<const uint32_t *>(keys);   // low word of key r at 2 r
    int32_t base = (int32_t)lo, len = (int32_t)(hi - lo);
    if (len <= 0) return -1;
    while (len > 1) {
        const int32_t half = len >> 1;
        base = alpha[2 * (int64_t)(base + half)] <= al ? base + half : base;
        len -= half;
    }
    return alpha[2 * (int64_t)base] == al ? (int64_t)base : -1;
}

// two searches of the same block in lockstep (two loads in flight per halving)
__device__ __forceinline__ void search_block2(const uint64_t *keys, int64_t lo, int64_t hi, uint32_t a0, uint32_t a1,
                                              int64_t &r0, int64_t &r1)
{
    const uint32_t *alpha = reinterpret_cast<const uint32_t *>(keys);
    int32_t b0 = (int32_t)lo, b1 = (int32_t)lo, len = (int32_t)(hi - lo);
    r0 = r1 = -1;
    if (len <= 0) return;
    while (len > 1) {
        const int32_t half = len >> 1;
        const uint32_t k0 = alpha[2 * (int64_t)(b0 + half)], k1 = alpha[2 * (int64_t)(b1 + half)];
        b0 = k0 <= a0 ? b0 + half : b0;
        b1 = k1 <= a1 ? b1 + half : b1;
        len -= half;
    }
    const uint32_t k0 = alpha[2 * (int64_t)b0], k1 = alpha[2 * (int64_t)b1];
    r0 = k0 == a0 ? (int64_t)b0 : -1;
    r1 = k1 == a1 ? (int64_t)b1 : -1;
}

template <int LK>
__device__ __forceinline__ int64_t find_row(const HamArgs &A, uint32_t al, uint32_t be)
{
    if constexpr (LK == kLkRanks) {
        return (int64_t)A.rankB[be] * A.nA + A.rankA[al];
    } else if constexpr (LK == kLkBlocks) {
        const int32_t b = A.bidx[be];
        if (b < 0) return -1;
        return search_block(A.keys, A.bstart[b], A.bstart[b + 1], al);
    } else {
        uint64_t key = (uint64_t)al | ((uint64_t)be << 32);
        const uint64_t hm = mix64h(key);
        // membership bitmap (a few MB, cache-resident) rejects most absent targets
        const uint64_t bit = hm >> (64 - A.hfbits);
        if (!((A.hfilter[bit >> 5] >> (bit & 31)) & 1u)) return -1;
        uint64_t slot = hm & A.hmask;
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
#ifndef IRL_SCAN_FACTOR
#define IRL_SCAN_FACTOR 8
#endif
constexpr int kScanFactor = IRL_SCAN_FACTOR;   // scan a block when it holds <= this many times the candidates it replaces
constexpr int kMaxPairs = 496;     // C(32, 2)

// one wavefront's lists in LDS, for at most MS single moves and MP orbital pairs per spin
template <int MS, int MP>
struct WaveListsT {
    uint32_t sA[MS];      // i | a << 5 | (sign < 0) << 10
    uint32_t sAstr[MS];
    uint32_t sB[MS];
    uint32_t sBstr[MS];
    uint16_t poA[MP], pvA[MP], poB[MP], pvB[MP];  // i | j << 8
    int32_t sBlo[MS], sBhi[MS];   // blocked lookup: rows of each beta single's target
    int32_t own_lo, own_hi;       // blocked lookup: rows sharing this row's beta
    int32_t alo, ahi;             // blocked lookup: alpha-major rows sharing its alpha
};
using WaveLists = WaveListsT<kMaxSingles, kMaxPairs>;   // any n <= 32 (10 KiB)
// n <= 20: na (n - na) <= 100 single moves and C(n, 2) <= 190 pairs.  At 4.5 KiB
// per wavefront the enumerating kernel's LDS no longer limits it to 4 wavefronts
// per SIMD.
constexpr int kSmallListsMaxN = 20;
using WaveListsSmall = WaveListsT<128, 192>;

// blocked lookup: row ranges of the beta-single targets and of the row's own beta
template <class WL>
__device__ void build_block_ranges(const HamArgs &A, WL &L, uint32_t al, uint32_t be, int lane)
{
    const int cnt = A.nb * (A.n - A.nb);
    for (int f = lane; f < cnt; f += kWave) {
        const int32_t b = A.bidx[L.sBstr[f]];
        L.sBlo[f] = b < 0 ? 0 : A.bstart[b];
        L.sBhi[f] = b < 0 ? 0 : A.bstart[b + 1];
    }
    if (lane == 0) {
        const int32_t b = A.bidx[be];
        L.own_lo = A.bstart[b];
        L.own_hi = A.bstart[b + 1];
        const int32_t a = A.aidx[al];
        L.alo = A.astart[a];
        L.ahi = A.astart[a + 1];
    }
}

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

// Visits p = lo + lane, lo + lane + stride, ... < hi with key(p) loaded four at a
// time, so that four loads are in flight before the first one is used; past hi the
// key is `none`, which the callers choose so that it matches no excitation.
template <typename LD, typename FN>
__device__ __forceinline__ void scan4(int64_t lo, int64_t hi, int lane, int stride, uint32_t none, LD key, FN fn)
{
    for (int64_t p0 = lo + lane; p0 < hi; p0 += 4 * (int64_t)stride) {
        uint32_t k[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t p = p0 + (int64_t)u * stride;
            k[u] = p < hi ? key(p) : none;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) fn(p0 + (int64_t)u * stride, k[u]);
    }
}

// Evaluate the candidates of one determinant on one lane (stride 64).  OP is
// called with (target row, sign, kind, value) for every target inside the set.
template <int LK, typename OP, class WL>
__device__ __forceinline__ void visit_row(const HamArgs &A, const WL &L, uint32_t al,
                                          uint32_t be, int lane, int stride, OP op)
{
    const int n = A.n, na = A.na, nb = A.nb, va = n - na, vb = n - nb;
    const uint32_t *alpha32 = reinterpret_cast<const uint32_t *>(A.keys);   // low word of key r at 2 r
    (void)alpha32;
    // Blocked lookup: a short own-beta block is scanned (its members that differ
    // from the row's alpha string by one or two orbitals are exactly the alpha
    // singles and alpha-alpha doubles inside the set) instead of probing every
    // candidate; likewise a short beta' block for the opposite-spin doubles.
    bool scan_own = false;
    if constexpr (LK == kLkBlocks) {
        const int cand = na * va + (na * (na - 1) / 2) * (va * (va - 1) / 2);
        scan_own = (L.own_hi - L.own_lo) <= kScanFactor * cand;
        if (scan_own) {
            scan4(L.own_lo, L.own_hi, lane, stride, al, [&](int64_t p) { return alpha32[2 * p]; },
                  [&](int64_t p, uint32_t a2) {
                const uint32_t x = al ^ a2;
                const int pc = __popc(x);
                if (pc == 2) {
                    const int i = __ffs(al & x) - 1, a = __ffs(a2 & x) - 1;
                    const int sg = move_sign(al, i, a);
                    op(p, sg, 1, sg * single_value(A.h, A.g, n, al, be, i, a));
                } else if (pc == 4) {
                    const uint32_t out = al & x, in = a2 & x;
                    const int i = __ffs(out) - 1, j = __ffs(out & (out - 1)) - 1;
                    const int a = __ffs(in) - 1, b = __ffs(in & (in - 1)) - 1;
                    const int s1 = move_sign(al, i, a);
                    const uint32_t b1 = (al & ~(1u << i)) | (1u << a);
                    const int s2 = move_sign(b1, j, b);
                    const double v = gint(A.g, n, i, a, j, b) - gint(A.g, n, i, b, j, a);
                    op(p, s1 * s2, 3, (s1 * s2) * v);
                }
            });
        }
    }
    // Blocked lookup, alpha side: the rows sharing this row's alpha string (its
    // alpha-major block) that differ in one or two beta orbitals are exactly the beta
    // singles and beta-beta doubles inside the set; a short block is scanned instead
    // of searching for each candidate.
    bool scan_alpha = false;
    if constexpr (LK == kLkBlocks) {
        const int cand = nb * vb + (nb * (nb - 1) / 2) * (vb * (vb - 1) / 2);
        scan_alpha = (L.ahi - L.alo) <= kScanFactor * cand;
        if (scan_alpha) {
            scan4(L.alo, L.ahi, lane, stride, be, [&](int64_t p) { return A.abeta[p]; },
                  [&](int64_t p, uint32_t b2) {
                const uint32_t x = be ^ b2;
                const int pc = __popc(x);
                if (pc == 2) {
                    const int i = __ffs(be & x) - 1, a = __ffs(b2 & x) - 1;
                    const int sg = move_sign(be, i, a);
                    op((int64_t)A.arow[p], sg, 2, sg * single_value(A.h, A.g, n, be, al, i, a));
                } else if (pc == 4) {
                    const uint32_t out = be & x, in = b2 & x;
                    const int i = __ffs(out) - 1, j = __ffs(out & (out - 1)) - 1;
                    const int a = __ffs(in) - 1, b = __ffs(in & (in - 1)) - 1;
                    const int s1 = move_sign(be, i, a);
                    const uint32_t b1 = (be & ~(1u << i)) | (1u << a);
                    const int s2 = move_sign(b1, j, b);
                    const double v = gint(A.g, n, i, a, j, b) - gint(A.g, n, i, b, j, a);
                    op((int64_t)A.arow[p], s1 * s2, 4, (s1 * s2) * v);
                }
            });
        }
    }
    // alpha and beta singles
    for (int spin = 0; spin < 2; ++spin) {
        if (spin == 0 && scan_own) continue;
        if (spin == 1 && scan_alpha) continue;
        const int cnt = spin ? nb * vb : na * va;
        const uint32_t *s = spin ? L.sB : L.sA;
        const uint32_t *ss = spin ? L.sBstr : L.sAstr;
        uint32_t same = spin ? be : al, other = spin ? al : be;
        for (int e = lane; e < cnt; e += stride) {
            uint32_t p = s[e];
            int i = p & 31, a = (p >> 5) & 31, sg = (p >> 10) & 1 ? -1 : 1;
            int64_t r;
            if constexpr (LK == kLkBlocks)
                r = spin ? search_block(A.keys, L.sBlo[e], L.sBhi[e], al)
                         : search_block(A.keys, L.own_lo, L.own_hi, ss[e]);
            else
                r = spin ? find_row<LK>(A, al, ss[e]) : find_row<LK>(A, ss[e], be);
            if (r >= 0) op(r, sg, spin ? 2 : 1, sg * single_value(A.h, A.g, n, same, other, i, a));
        }
    }
    // same-spin doubles
    for (int spin = 0; spin < 2; ++spin) {
        if (spin == 0 && scan_own) continue;
        if (spin == 1 && scan_alpha) continue;
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
            int64_t r;
            if constexpr (LK == kLkBlocks)
                r = spin ? find_row<LK>(A, al, b2) : search_block(A.keys, L.own_lo, L.own_hi, b2);
            else
                r = spin ? find_row<LK>(A, al, b2) : find_row<LK>(A, b2, be);
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
    if constexpr (LK == kLkBlocks) {
        const int cA = na * va, cB = nb * vb;
        for (int f = 0; f < cB && cA > 0; ++f) {
            const int32_t lo = L.sBlo[f], hi = L.sBhi[f];
            if (hi <= lo) continue;
            const uint32_t pb = L.sB[f];
            const int j = pb & 31, b = (pb >> 5) & 31, sgb = (pb >> 10) & 1 ? -1 : 1;
            if (hi - lo <= kScanFactor * cA) {
                scan4(lo, hi, lane, stride, al, [&](int64_t p) { return alpha32[2 * p]; },
                      [&](int64_t p, uint32_t a2) {
                    const uint32_t x = al ^ a2;
                    if (__popc(x) != 2) return;
                    const int i = __ffs(al & x) - 1, a = __ffs(a2 & x) - 1;
                    const int sg = move_sign(al, i, a) * sgb;
                    op(p, sg, 5, sg * gint(A.g, n, i, a, j, b));
                });
            } else {
                // two alpha singles per lane and pass, searched together; the second
                // of a pair past cA searches the first's string and is not used
                for (int xa = lane; xa < cA; xa += 2 * stride) {
                    const int xb = xa + stride < cA ? xa + stride : xa;
                    int64_t ra, rb;
                    search_block2(A.keys, lo, hi, L.sAstr[xa], L.sAstr[xb], ra, rb);
                    if (ra >= 0) {
                        const uint32_t pa = L.sA[xa];
                        const int i = pa & 31, a = (pa >> 5) & 31;
                        const int sg = ((pa >> 10) & 1 ? -1 : 1) * sgb;
                        op(ra, sg, 5, sg * gint(A.g, n, i, a, j, b));
                    }
                    if (xa + stride < cA && rb >= 0) {
                        const uint32_t pa = L.sA[xb];
                        const int i = pa & 31, a = (pa >> 5) & 31;
                        const int sg = ((pa >> 10) & 1 ? -1 : 1) * sgb;
                        op(rb, sg, 5, sg * gint(A.g, n, i, a, j, b));
                    }
                }
            }
        }
    } else {
        const int cA = na * va, cB = nb * vb, cnt = cA * cB;
        if (cnt > 0) {
            int xa = lane / cB, xb = lane - xa * cB;
            const int step_a = stride / cB, step_b = stride - step_a * cB;
            for (int e = lane; e < cnt; e += stride) {
                uint32_t pa = L.sA[xa], pb = L.sB[xb];
                int i = pa & 31, a = (pa >> 5) & 31, j = pb & 31, b = (pb >> 5) & 31;
                int sg = (((pa >> 10) ^ (pb >> 10)) & 1) ? -1 : 1;
                const int64_t r = find_row<LK>(A, L.sAstr[xa], L.sBstr[xb]);
                if (r >= 0) op(r, sg, 5, sg * gint(A.g, n, i, a, j, b));
                xb += step_b;
                xa += step_a;
                if (xb >= cB) { xb -= cB; ++xa; }
            }
        }
    }
}

// one determinant row on one wavefront: u[row] = H_rr w[row] + sum of the row's connections
// lists of one row's single moves and pairs (and, for the blocked lookup, the
// row ranges of its beta-single targets), written by the 64 lanes of its wave
template <int LK, class WL>
__device__ __forceinline__ void prepare_row(const HamArgs &A, WL &L, uint32_t al, uint32_t be,
                                            int lane)
{
    build_lists(al, A.n, A.na, L.sA, L.sAstr, L.poA, L.pvA, lane);
    build_lists(be, A.n, A.nb, L.sB, L.sBstr, L.poB, L.pvB, lane);
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if constexpr (LK == kLkBlocks) {
        build_block_ranges(A, L, al, be, lane);
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
}

__device__ __forceinline__ void end_row()
{
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int LK, class WL>
__device__ __forceinline__ void pull_row(const HamArgs &A, WL &L, int64_t row, int lane,
                                         const double *__restrict__ w, double *__restrict__ u)
{
    uint64_t key = A.keys[row];
    uint32_t al = (uint32_t)key, be = (uint32_t)(key >> 32);
    prepare_row<LK>(A, L, al, be, lane);
    double acc = 0.0;
    visit_row<LK>(A, L, al, be, lane, kWave,
                    [&](int64_t r, int, int, double v) { acc += v * w[r]; });
    acc = wave_sum(acc);
    if (lane == 0) u[row] = A.diag[row] * w[row] + acc;
    end_row();
}

// rows [r0, r1), one wavefront per row, NW wavefronts per workgroup, grid-stride.
// With the small lists, LDS allows 8 wavefronts per SIMD; the launch bound asks the
// compiler for registers to match (some scalar registers then live in vector lanes).
template <int LK, int NW = 4, class WL = WaveLists>
__global__ __launch_bounds__(64 * NW, sizeof(WL) <= 8192 ? 8 : 4) void k_ham_pull(HamArgs A, const double *__restrict__ w,
                                                      double *__restrict__ u, int64_t r0, int64_t r1)
{
    __shared__ WL lists[NW];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t nwaves = (int64_t)gridDim.x * NW;
    for (int64_t row = r0 + (int64_t)blockIdx.x * NW + wv; row < r1; row += nwaves)
        pull_row<LK>(A, lists[wv], row, lane, w, u);
}

template <int LK, class WL>
static void launch_pull_lists(const HamArgs &A, const double *w, double *u, int64_t r0, int64_t r1, int nw,
                              int64_t cap, hipStream_t st)
{
    int64_t blocks = (r1 - r0 + nw - 1) / nw;
    if (blocks > cap) blocks = cap;
    if (nw == 1)
        k_ham_pull<LK, 1, WL><<<(unsigned)blocks, 64, 0, st>>>(A, w, u, r0, r1);
    else if (nw == 2)
        k_ham_pull<LK, 2, WL><<<(unsigned)blocks, 128, 0, st>>>(A, w, u, r0, r1);
    else
        k_ham_pull<LK, 4, WL><<<(unsigned)blocks, 256, 0, st>>>(A, w, u, r0, r1);
}

template <int LK>
static void launch_pull(const HamArgs &A, const double *w, double *u, int64_t r0, int64_t r1, int nw, int64_t cap,
                        hipStream_t st)
{
    if (A.n <= kSmallListsMaxN)
        launch_pull_lists<LK, WaveListsSmall>(A, w, u, r0, r1, nw, cap, st);
    else
        launch_pull_lists<LK, WaveLists>(A, w, u, r0, r1, nw, cap, st);
}

// Stored rows: u[row] = diag * w[row] + sum_p val[p] w[col[p]], one wave per row.
// The elements of a row are split into column blocks (targets [b 2^hcs, (b + 1)
// 2^hcs), a slice of w that stays in L2) and each block is its own launch, so the
// random gathers of every XCD hit one resident slice; u accumulates over the
// blocks in block order.  The elements are streamed once per apply (non-temporal);
// each lane keeps four gathers of w in flight.  Lane partial sums are combined by
// a fixed butterfly, so the result does not depend on scheduling.
__device__ __forceinline__ double stored_block_sum(const HamArgs &A, int b, int64_t row, int lane,
                                                   const double *__restrict__ w)
{
    const int64_t *ptr = A.hptr + (int64_t)b * (A.ns + 1);
    const int64_t p1 = ptr[row + 1];
    int64_t p = ptr[row] + lane;
    double acc = 0.0;
    for (; p + 3 * kWave < p1; p += 4 * kWave) {
        int32_t c[4];
        double v[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            c[q] = __builtin_nontemporal_load(A.hcol + p + q * kWave);
            v[q] = __builtin_nontemporal_load(A.hval + p + q * kWave);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) acc += v[q] * w[c[q]];
    }
    for (; p < p1; p += kWave)
        acc += __builtin_nontemporal_load(A.hval + p) * w[__builtin_nontemporal_load(A.hcol + p)];
    return wave_sum(acc);
}

// u[row] after column block b: fma(diag, w, S_0) for b = 0, then + S_b
__device__ __forceinline__ double stored_accumulate(const HamArgs &A, int b, int64_t row, double prev,
                                                    double acc, const double *__restrict__ w)
{
    return b == 0 ? fma(A.diag[row], w[row], acc) : prev + acc;
}

// all column blocks of one row in block order (the grouped launch)
__device__ __forceinline__ void stored_row(const HamArgs &A, int64_t row, int lane, const double *__restrict__ w,
                                           double *__restrict__ u)
{
    double t = 0.0;
    for (int b = 0; b < A.hcb; ++b) t = stored_accumulate(A, b, row, t, stored_block_sum(A, b, row, lane, w), w);
    if (lane == 0) u[row] = t;
}

__global__ __launch_bounds__(256) void k_ham_stored(HamArgs A, const double *__restrict__ w,
                                                    double *__restrict__ u, int64_t r0, int64_t r1, int b)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t nwaves = (int64_t)gridDim.x * 4;
    for (int64_t row = r0 + (int64_t)blockIdx.x * 4 + wv; row < r1; row += nwaves) {
        const double acc = stored_block_sum(A, b, row, lane, w);
        if (lane == 0) u[row] = stored_accumulate(A, b, row, b == 0 ? 0.0 : u[row], acc, w);
    }
}

// Stored rows, first pass: number of connections of each row inside the set, per
// column block (count[b ns + row]).
template <int LK>
__global__ __launch_bounds__(256) void k_ham_count(HamArgs A, int32_t *__restrict__ count)
{
    __shared__ WaveLists lists[4];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t nwaves = (int64_t)gridDim.x * 4;
    for (int64_t row = (int64_t)blockIdx.x * 4 + wv; row < A.ns; row += nwaves) {
        uint64_t key = A.keys[row];
        uint32_t al = (uint32_t)key, be = (uint32_t)(key >> 32);
        prepare_row<LK>(A, lists[wv], al, be, lane);
        int c[kMaxColBlocks];
#pragma unroll
        for (int bb = 0; bb < kMaxColBlocks; ++bb) c[bb] = 0;
        visit_row<LK>(A, lists[wv], al, be, lane, kWave, [&](int64_t r, int, int, double) {
            const int b = (int)(r >> A.hcs);
#pragma unroll
            for (int bb = 0; bb < kMaxColBlocks; ++bb) c[bb] += b == bb;
        });
#pragma unroll
        for (int bb = 0; bb < kMaxColBlocks; ++bb) {
            for (int off = 32; off > 0; off >>= 1) c[bb] += __shfl_xor(c[bb], off, kWave);
            if (lane == 0 && bb < A.hcb) count[(int64_t)bb * A.ns + row] = c[bb];
        }
        end_row();
    }
}

// Stored rows, second pass: each lane counts its own connections per column block
// again, an exclusive scan over the lanes gives its first slot in each block, and
// a third enumeration writes them.  The layout inside a row's block is therefore
// fixed (lane-major), and writes never leave [ptr_b[row], ptr_b[row + 1]).
template <int LK>
__global__ __launch_bounds__(256) void k_ham_fill(HamArgs A, const int64_t *__restrict__ ptr,
                                                  int32_t *__restrict__ col, double *__restrict__ val)
{
    __shared__ WaveLists lists[4];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t nwaves = (int64_t)gridDim.x * 4;
    for (int64_t row = (int64_t)blockIdx.x * 4 + wv; row < A.ns; row += nwaves) {
        uint64_t key = A.keys[row];
        uint32_t al = (uint32_t)key, be = (uint32_t)(key >> 32);
        prepare_row<LK>(A, lists[wv], al, be, lane);
        int c[kMaxColBlocks];
#pragma unroll
        for (int bb = 0; bb < kMaxColBlocks; ++bb) c[bb] = 0;
        visit_row<LK>(A, lists[wv], al, be, lane, kWave, [&](int64_t r, int, int, double) {
            const int b = (int)(r >> A.hcs);
#pragma unroll
            for (int bb = 0; bb < kMaxColBlocks; ++bb) c[bb] += b == bb;
        });
        int64_t pos[kMaxColBlocks], end[kMaxColBlocks];
#pragma unroll
        for (int bb = 0; bb < kMaxColBlocks; ++bb) {
            int incl = c[bb];
            for (int off = 1; off < kWave; off <<= 1) {
                const int t = __shfl_up(incl, off, kWave);
                if (lane >= off) incl += t;
            }
            const int64_t *pb = ptr + (int64_t)(bb < A.hcb ? bb : 0) * (A.ns + 1);
            pos[bb] = bb < A.hcb ? pb[row] + (incl - c[bb]) : 0;
            end[bb] = bb < A.hcb ? pb[row + 1] : 0;
        }
        visit_row<LK>(A, lists[wv], al, be, lane, kWave, [&](int64_t r, int, int, double v) {
            const int b = (int)(r >> A.hcs);
#pragma unroll
            for (int bb = 0; bb < kMaxColBlocks; ++bb) {
                if (b == bb) {
                    if (pos[bb] < end[bb]) {
                        col[pos[bb]] = (int32_t)r;
                        val[pos[bb]] = v;
                    }
                    ++pos[bb];
                }
            }
        });
        end_row();
    }
}

// ---- stored rows, LDS-sliced layout ---------------------------------------------
// For sets larger than an L2-resident slice of w, the targets are split into
// slices of 2^scs rows whose w (128 KiB) one workgroup stages in LDS, so the
// random gathers of w become LDS reads and HBM streams only the elements.  Inside
// a slice, rows are ordered by their element count within windows of kSellWindow
// rows and grouped 64 per wavefront (one row per lane); a group of longest row L
// holds L x 64 slots, slot (j, lane) the j-th element of the lane's row (zero
// padding past its end), as a 16-bit target inside the slice and an FP64 value.

// first pass: connections of each row inside each slice (count[b ns + row])
template <int LK, class WL>
__global__ __launch_bounds__(256) void k_ham_count_sliced(HamArgs A, int scs, int scb, uint32_t *__restrict__ count)
{
    __shared__ WL lists[4];
    __shared__ uint32_t cnt[4][kMaxSlices];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t nwaves = (int64_t)gridDim.x * 4;
    for (int64_t row = (int64_t)blockIdx.x * 4 + wv; row < A.ns; row += nwaves) {
        for (int b = lane; b < scb; b += kWave) cnt[wv][b] = 0u;
        const uint64_t key = A.keys[row];
        const uint32_t al = (uint32_t)key, be = (uint32_t)(key >> 32);
        prepare_row<LK>(A, lists[wv], al, be, lane);
        visit_row<LK>(A, lists[wv], al, be, lane, kWave, [&](int64_t r, int, int, double) {
            atomicAdd(&cnt[wv][(int)(r >> scs)], 1u);
        });
        end_row();
        for (int b = lane; b < scb; b += kWave) count[(int64_t)b * A.ns + row] = cnt[wv][b];
        end_row();
    }
}

// Slot (j, lane) of a group (j < L, L even) inside the group's slot range: values
// and targets in lane-interleaved pairs (a lane loads the 16 bytes of values or
// the 4 bytes of targets of slots 2i and 2i + 1), so a wavefront's loads are 1 KiB
// of values and 256 bytes of targets.
__host__ __device__ __forceinline__ int64_t sell_val_slot(int64_t j, int64_t lane)
{
    return (j >> 1) * (2 * kWave) + lane * 2 + (j & 1);
}

__host__ __device__ __forceinline__ int64_t sell_col_slot(int64_t j, int64_t lane)
{
    return (j >> 1) * (2 * kWave) + lane * 2 + (j & 1);
}

// second pass, one wavefront per workgroup: each lane counts its own connections
// per slice (LDS table [lane][slice], sized for the set's slices at launch, with an
// odd row stride so that the lanes' entries of one slice fall in distinct banks),
// an exclusive scan over the lanes gives each
// lane's first position j in the row's run of each slice, and a second enumeration
// writes element j of (slice b, row) to slots sell_val_slot / sell_col_slot (j, lane) of the row's group
// and lane (slot[b][row] = group * 64 + lane): the layout, and so the apply's
// summation order, are fixed by the set.
template <int LK, class WL>
__global__ __launch_bounds__(64) void k_ham_fill_sliced(HamArgs A, int scs, int scb, int cs,
                                                        const int64_t *__restrict__ sbase,
                                                        const uint32_t *__restrict__ sgbase, int sgroups,
                                                        const uint16_t *__restrict__ sglen,
                                                        const uint32_t *__restrict__ slot,
                                                        uint16_t *__restrict__ scol, double *__restrict__ sval)
{
    __shared__ WL lists;
    extern __shared__ uint32_t cnt_tab[];   // [kWave][cs], cs >= scb
    auto cnt = [&](int l, int b) -> uint32_t & { return cnt_tab[l * cs + b]; };
    const int lane = threadIdx.x;
    const uint32_t mask = (1u << scs) - 1u;
    for (int64_t row = blockIdx.x; row < A.ns; row += gridDim.x) {
        for (int b = 0; b < scb; ++b) cnt(lane, b) = 0u;
        const uint64_t key = A.keys[row];
        const uint32_t al = (uint32_t)key, be = (uint32_t)(key >> 32);
        prepare_row<LK>(A, lists, al, be, lane);
        visit_row<LK>(A, lists, al, be, lane, kWave, [&](int64_t r, int, int, double) {
            ++cnt(lane, (int)(r >> scs));
        });
        end_row();
        // lane b (and b + 64, ...) turns column b of the table into first positions
        for (int b = lane; b < scb; b += kWave) {
            uint32_t run = 0u;
            for (int l = 0; l < kWave; ++l) {
                const uint32_t c = cnt(l, b);
                cnt(l, b) = run;
                run += c;
            }
        }
        end_row();
        visit_row<LK>(A, lists, al, be, lane, kWave, [&](int64_t r, int, int, double v) {
            const int b = (int)(r >> scs);
            const uint32_t j = cnt(lane, b)++;
            const uint32_t sl = slot[(int64_t)b * A.ns + row];
            const int64_t g = (int64_t)b * sgroups + (sl >> 6);
            if (j < sglen[g]) {
                const int64_t p0 = sbase[b] + sgbase[g], lane_s = sl & 63u;
                scol[p0 + sell_col_slot(j, lane_s)] = (uint16_t)((uint32_t)r & mask);
                sval[p0 + sell_val_slot(j, lane_s)] = v;
            }
        });
        end_row();
    }
}

hipError_t launch_ham_count_sliced(const irl_system *s, int scs, int scb, uint32_t *count, hipStream_t st)
{
    HamArgs A = ham_view(s);
    int64_t blocks = (s->ns + 3) / 4;
    if (blocks > 65536) blocks = 65536;
    if (scb < 1 || scb > kMaxSlices) return hipErrorInvalidValue;
    const bool small = s->n <= kSmallListsMaxN;
    if (s->lookup == kLkBlocks) {
        if (small) k_ham_count_sliced<kLkBlocks, WaveListsSmall><<<(unsigned)blocks, 256, 0, st>>>(A, scs, scb, count);
        else k_ham_count_sliced<kLkBlocks, WaveLists><<<(unsigned)blocks, 256, 0, st>>>(A, scs, scb, count);
    } else if (s->lookup == kLkHash) {
        if (small) k_ham_count_sliced<kLkHash, WaveListsSmall><<<(unsigned)blocks, 256, 0, st>>>(A, scs, scb, count);
        else k_ham_count_sliced<kLkHash, WaveLists><<<(unsigned)blocks, 256, 0, st>>>(A, scs, scb, count);
    } else {
        if (small) k_ham_count_sliced<kLkRanks, WaveListsSmall><<<(unsigned)blocks, 256, 0, st>>>(A, scs, scb, count);
        else k_ham_count_sliced<kLkRanks, WaveLists><<<(unsigned)blocks, 256, 0, st>>>(A, scs, scb, count);
    }
    return hipGetLastError();
}

template <int LK, class WL>
static void launch_fill_sliced_lists(const irl_system *s, const HamArgs &A, int64_t blocks, int scs, int scb, int cs,
                                     const uint32_t *slot, uint16_t *scol, double *sval, hipStream_t st)
{
    const size_t lds = (size_t)kWave * cs * sizeof(uint32_t);
    k_ham_fill_sliced<LK, WL><<<(unsigned)blocks, 64, lds, st>>>(A, scs, scb, cs, s->d.sbase, s->d.sgbase,
                                                                 s->d.sgroups, s->d.sglen, slot, scol, sval);
}

hipError_t launch_ham_fill_sliced(const irl_system *s, int scs, int scb, const uint32_t *slot, uint16_t *scol,
                                  double *sval, hipStream_t st)
{
    HamArgs A = ham_view(s);
    int64_t blocks = s->ns;
    if (blocks > 262144) blocks = 262144;
    if (scb < 1 || scb > kMaxSlices) return hipErrorInvalidValue;
    // odd row stride of the per-lane count table while it stays within 64 KiB
    const int cs = (scb | 1) * kWave * 4 <= 65536 ? (scb | 1) : scb;
    const bool small = s->n <= kSmallListsMaxN;
    if (s->lookup == kLkBlocks) {
        if (small) launch_fill_sliced_lists<kLkBlocks, WaveListsSmall>(s, A, blocks, scs, scb, cs, slot, scol, sval, st);
        else launch_fill_sliced_lists<kLkBlocks, WaveLists>(s, A, blocks, scs, scb, cs, slot, scol, sval, st);
    } else if (s->lookup == kLkHash) {
        if (small) launch_fill_sliced_lists<kLkHash, WaveListsSmall>(s, A, blocks, scs, scb, cs, slot, scol, sval, st);
        else launch_fill_sliced_lists<kLkHash, WaveLists>(s, A, blocks, scs, scb, cs, slot, scol, sval, st);
    } else {
        if (small) launch_fill_sliced_lists<kLkRanks, WaveListsSmall>(s, A, blocks, scs, scb, cs, slot, scol, sval, st);
        else launch_fill_sliced_lists<kLkRanks, WaveLists>(s, A, blocks, scs, scb, cs, slot, scol, sval, st);
    }
    return hipGetLastError();
}

// Apply of the sliced layout: k_ham_sell_win sums each row's elements slice by slice
// (below), k_ham_sliced_sum adds the partial sums of the runs of slices when a window's
// slices are split into runs.
#ifndef IRL_SELL_UNROLL
#define IRL_SELL_UNROLL 16
#endif
constexpr int kSellUnroll = IRL_SELL_UNROLL;
// word 3 of a raw buffer descriptor on gfx9-family parts: 32-bit data format, no
// swizzle, no index stride; with stride 0 the size (word 2) is in bytes and loads at
// or past it return zeros
constexpr int kBufferWord3 = 0x00020000;
// cache policy of the streamed loads: non-temporal (the stored rows are read once per
// apply, so they should not displace w, the lane rows or the partial sums in L2)
constexpr int kStreamPolicy = 2;

// k_ham_sell_win: a workgroup owns one window of 4096 rows and a run of consecutive
// slices.  For each slice it stages the slice's w (128 KiB) in LDS; its 16 wavefronts
// then take the window's 64 groups of that slice, 4 each: wavefront wv's k-th group is
// 16 k + wv for even k and 16 k + 15 - wv for odd k (groups run from long to short
// inside a window, so alternating directions evens out the work).  A wavefront's
// groups form one stream of chunks of 16 slots (8 KiB of values and 2 KiB of targets,
// both as lane pairs); the next chunk's loads are issued before the current one
// is summed.  Each chunk reads through buffer descriptors whose size ends at its
// group's end: pairs past the end read as zeros (values 0, targets 0) without touching
// memory, so every chunk issues the same loads and the waits before a sum count only
// that chunk's loads.  Lane l of a group sums its row's elements (targets index the
// LDS copy of w) and adds the sum to the row's accumulator in LDS: a row occurs once
// per slice, so no two lanes touch one accumulator within a slice, and slices are
// separated by barriers, so every row sums its slices in slice order.  At the end the
// workgroup writes u = H_rr w + sum when it owns all slices, else the run's partial
// sum, which k_ham_sliced_sum adds over the runs in order.  No per-slice partial sum
// reaches memory.
constexpr int kWinThreads = 1024;
constexpr int kWinGroups = kSellWindow / kWave;   // groups per window (64)

__global__ __launch_bounds__(kWinThreads) void k_ham_sell_win(HamArgs A, const double *__restrict__ w,
                                                              double *__restrict__ u, int64_t r0, int64_t r1,
                                                              int64_t wa, int spg)
{
    constexpr int SL = 1 << kSliceLog, PER = SL / (2 * kWinThreads), K = kSellUnroll, NW = kWinThreads / kWave;
    constexpr int GPW = kWinGroups / NW;   // groups of a wavefront per slice
    static_assert(GPW <= kWave, "one group of a wavefront's share per lane");
    __shared__ double wl[SL];
    __shared__ double acc[kSellWindow];
    const int t = threadIdx.x, lane = t & 63;
    const int wv = __builtin_amdgcn_readfirstlane(t >> 6);
    const int64_t win = wa + blockIdx.x;
    const int sg = blockIdx.y;
    const int b0 = sg * spg, b1 = min(A.scb, b0 + spg);
    const int64_t gw0 = win * kWinGroups;
    const int ngw = (int)min((int64_t)kWinGroups, (int64_t)A.sgroups - gw0);
    for (int i = t; i < kSellWindow; i += kWinThreads) acc[i] = 0.0;
    auto group_of = [&](int kk) { return kk * NW + ((kk & 1) ? NW - 1 - wv : wv); };
    static_assert(K == 16, "chunk offsets below assume 16 slots");
    const int vo0 = lane * 16, vo1 = lane * 16 + 4096, co = lane * 4, po = lane * 2;
    struct Chunk {
        double2 v[K / 2];
        uint32_t c[K / 2];
        uint32_t lr;
    };
    for (int b = b0; b < b1; ++b) {
        // every wavefront is done with the previous slice's copy of w
        __syncthreads();
        const int64_t c0 = (int64_t)b << A.scs;
        const int nc = (int)min((int64_t)SL, A.ns - c0);
        const int64_t gb = (int64_t)b * A.sgroups + gw0;   // the window's first group in slice b
        // the wavefront's groups of this slice: lane k < GPW keeps group k's slot
        // offset and length
        uint32_t mbase = 0, mlen = 0;
        if (lane < GPW) {
            const int gi = group_of(lane);
            if (gi < ngw) {
                mbase = A.sgbase[gb + gi];
                mlen = A.sglen[gb + gi];
            }
        }
        if (nc == SL) {
            double2 x[PER];
#pragma unroll
            for (int j = 0; j < PER; ++j) x[j] = *reinterpret_cast<const double2 *>(w + c0 + 2 * (t + j * kWinThreads));
#pragma unroll
            for (int j = 0; j < PER; ++j) {
                wl[2 * (t + j * kWinThreads)] = x[j].x;
                wl[2 * (t + j * kWinThreads) + 1] = x[j].y;
            }
        } else {
            for (int i = t; i < nc; i += kWinThreads) wl[i] = w[c0 + i];
        }
        __syncthreads();
        const uint64_t sb64 = (uint64_t)A.sbase[b];
        const int64_t sb = (int64_t)(((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(sb64 >> 32)) << 32) |
                                     (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)sb64));
        const uint16_t *col = A.scol + sb;
        const double *val = A.sval + sb;
        const __amdgpu_buffer_rsrc_t prs =
            __builtin_amdgcn_make_buffer_rsrc((void *)(A.sperm + gb * kWave), 0, ngw * kWave * 2, kBufferWord3);
        auto load = [&](Chunk &x, uint32_t base, int j0, int L, int gi) {
            const int left = L - j0;
            const __amdgpu_buffer_rsrc_t vrs = __builtin_amdgcn_make_buffer_rsrc(
                (void *)(val + base + (uint32_t)j0 * kWave), 0, left * kWave * 8, kBufferWord3);
            const __amdgpu_buffer_rsrc_t crs = __builtin_amdgcn_make_buffer_rsrc(
                (void *)(col + base + (uint32_t)j0 * kWave), 0, left * kWave * 2, kBufferWord3);
            x.lr = __builtin_amdgcn_raw_buffer_load_b16(prs, po, gi * kWave * 2, 0);
#pragma unroll
            for (int k = 0; k < K / 2; ++k) {
                const auto r = __builtin_amdgcn_raw_buffer_load_b128(
                    vrs, k < 4 ? vo0 + k * 1024 : vo1 + (k - 4) * 1024, 0, kStreamPolicy);
                x.v[k] = double2{__builtin_bit_cast(double, (uint64_t)r[0] | ((uint64_t)r[1] << 32)),
                                 __builtin_bit_cast(double, (uint64_t)r[2] | ((uint64_t)r[3] << 32))};
            }
#pragma unroll
            for (int q = 0; q < K / 2; ++q)
                x.c[q] = __builtin_amdgcn_raw_buffer_load_b32(crs, co + q * 256, 0, kStreamPolicy);
        };
        auto sum = [&](const Chunk &x, double a) {
#pragma unroll
            for (int q = 0; q < K / 2; ++q) {
                a += x.v[q].x * wl[x.c[q] & 0xffffu];
                a += x.v[q].y * wl[x.c[q] >> 16];
            }
            return a;
        };
        int i = group_of(0), k = 0;
        if (i < ngw) {
            int L = __builtin_amdgcn_readlane((int)mlen, 0);
            uint32_t base = (uint32_t)__builtin_amdgcn_readlane((int)mbase, 0);
            int j0 = 0;
            double gs = 0.0;
            Chunk ca, cb;
            load(ca, base, 0, L, i);
            auto step = [&](Chunk &cur, Chunk &nxt) -> bool {
                const bool last = j0 + K >= L;
                const int kn = min(k + 1, GPW - 1);
                const int gL = __builtin_amdgcn_readlane((int)mlen, kn);
                const uint32_t gbase = (uint32_t)__builtin_amdgcn_readlane((int)mbase, kn);
                const int ni = last ? (k + 1 < GPW ? group_of(k + 1) : ngw) : i, nj = last ? 0 : j0 + K;
                const int nL = last ? gL : L;
                const uint32_t nbase = last ? gbase : base;
                const bool more = ni < ngw;
                load(nxt, more ? nbase : base, more ? nj : j0, more ? nL : L, more ? ni : i);
                gs = sum(cur, gs);
                if (last) {
                    const uint32_t lr = cur.lr;
                    if (lr != 0xffffu) acc[lr] += gs;
                    gs = 0.0;
                }
                k = last ? k + 1 : k;
                i = ni;
                j0 = nj;
                L = nL;
                base = nbase;
                return more;
            };
            while (step(ca, cb) && step(cb, ca)) {
            }
        }
    }
    __syncthreads();
    const int64_t row0 = win * kSellWindow;
    const bool whole = b0 == 0 && b1 == A.scb;
    double *part = A.spart + (int64_t)sg * A.ns;
    for (int i = t; i < kSellWindow; i += kWinThreads) {
        const int64_t row = row0 + i;
        if (row < r0 || row >= r1) continue;
        if (whole)
            u[row] = fma(A.diag[row], w[row], acc[i]);
        else
            part[row] = acc[i];
    }
}

// u[row] = H_rr w[row] + sum over the nparts partial sums in order
__global__ __launch_bounds__(256) void k_ham_sliced_sum(HamArgs A, const double *__restrict__ w,
                                                        double *__restrict__ u, int64_t r0, int64_t r1, int nparts)
{
    const int64_t row = r0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (row >= r1) return;
    double acc = 0.0;
    for (int b = 0; b < nparts; ++b) acc += A.spart[(int64_t)b * A.ns + row];
    u[row] = fma(A.diag[row], w[row], acc);
}

#ifndef IRL_SELL_WIN_GOAL
#define IRL_SELL_WIN_GOAL 512
#endif
// window-major workgroups wanted for the whole set: with fewer windows than this a
// window's slices are split into runs, each adding one partial sum per row (two
// workgroups per CU balance the windows' unequal work; more runs only add partial
// sums).  The run count depends on the set alone, so a row's sum does not depend on
// the row range of the launch.
constexpr int kSellWinGoal = IRL_SELL_WIN_GOAL;

static hipError_t launch_ham_sliced(const irl_system *s, const HamArgs &A, const double *w, double *u, int64_t r0,
                                    int64_t r1, hipStream_t st)
{
    (void)s;
    const int64_t windows = (A.ns + kSellWindow - 1) / kSellWindow;
    int runs = (int)((kSellWinGoal + windows - 1) / windows);
    if (runs < 1) runs = 1;
    if (runs > A.scb) runs = A.scb;
    const int spg = (A.scb + runs - 1) / runs;
    runs = (A.scb + spg - 1) / spg;
    const int64_t wa = r0 / kSellWindow, wz = (r1 + kSellWindow - 1) / kSellWindow;
    k_ham_sell_win<<<dim3((unsigned)(wz - wa), (unsigned)runs), kWinThreads, 0, st>>>(A, w, u, r0, r1, wa, spg);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || runs == 1) return e;
    k_ham_sliced_sum<<<(unsigned)((r1 - r0 + 255) / 256), 256, 0, st>>>(A, w, u, r0, r1, runs);
    return hipGetLastError();
}

// Grouped H rows: one block per 4-row group, as in the solo launch.  Item k
// = (member m, first block a, b row groups); the items are in ascending a, and
// each block finds its item by a binary search (uniform, scalar loads).
// which = 0: w -> u, 1: psi -> H psi.
__device__ __forceinline__ int find_item(const WorkItem *__restrict__ items, int nitems, int blk)
{
    int lo = 0, hi = nitems - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (items[mid].a <= blk) lo = mid; else hi = mid - 1;
    }
    return lo;
}

template <int LK, class WL>
__global__ __launch_bounds__(256, sizeof(WL) <= 8192 ? 8 : 4) void k_ham_pull_grouped(
    const Member *__restrict__ M, const WorkItem *__restrict__ items, int nitems, int which)
{
    __shared__ WL lists[4];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const WorkItem it = items[find_item(items, nitems, (int)blockIdx.x)];
    const Member &mb = M[it.m];
    const double *w = which ? mb.psi : mb.w;
    double *u = which ? mb.hpsi : mb.u;
    const int64_t row = 4 * (int64_t)((int)blockIdx.x - it.a) + wv;
    if (row < mb.ns) pull_row<LK>(mb.ham, lists[wv], row, lane, w, u);
}

__global__ __launch_bounds__(256) void k_ham_stored_grouped(const Member *__restrict__ M,
                                                            const WorkItem *__restrict__ items,
                                                            int nitems, int which)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const WorkItem it = items[find_item(items, nitems, (int)blockIdx.x)];
    const Member &mb = M[it.m];
    const double *w = which ? mb.psi : mb.w;
    double *u = which ? mb.hpsi : mb.u;
    const int64_t row = 4 * (int64_t)((int)blockIdx.x - it.a) + wv;
    if (row < mb.ns) stored_row(mb.ham, row, lane, w, u);
}

hipError_t launch_ham_stored_grouped(const Member *M, const WorkItem *items, int nitems,
                                     int64_t nblocks, int which, hipStream_t st)
{
    if (nitems <= 0 || nblocks <= 0) return hipSuccess;
    k_ham_stored_grouped<<<(unsigned)nblocks, 256, 0, st>>>(M, items, nitems, which);
    return hipGetLastError();
}

hipError_t launch_ham_pull_grouped(const Member *M, const WorkItem *items, int nitems,
                                   int64_t nblocks, int which, int lookup, int max_n, hipStream_t st)
{
    if (nitems <= 0 || nblocks <= 0) return hipSuccess;
    // small lists when every member has n <= 20 (the same sums: only LDS sizes differ)
    if (lookup == kLkBlocks) {
        if (max_n <= kSmallListsMaxN)
            k_ham_pull_grouped<kLkBlocks, WaveListsSmall><<<(unsigned)nblocks, 256, 0, st>>>(M, items, nitems, which);
        else
            k_ham_pull_grouped<kLkBlocks, WaveLists><<<(unsigned)nblocks, 256, 0, st>>>(M, items, nitems, which);
    } else if (lookup == kLkHash) {
        if (max_n <= kSmallListsMaxN)
            k_ham_pull_grouped<kLkHash, WaveListsSmall><<<(unsigned)nblocks, 256, 0, st>>>(M, items, nitems, which);
        else
            k_ham_pull_grouped<kLkHash, WaveLists><<<(unsigned)nblocks, 256, 0, st>>>(M, items, nitems, which);
    } else {
        if (max_n <= kSmallListsMaxN)
            k_ham_pull_grouped<kLkRanks, WaveListsSmall><<<(unsigned)nblocks, 256, 0, st>>>(M, items, nitems, which);
        else
            k_ham_pull_grouped<kLkRanks, WaveLists><<<(unsigned)nblocks, 256, 0, st>>>(M, items, nitems, which);
    }
    return hipGetLastError();
}

HamView ham_view(const irl_system *s)
{
    HamArgs A;
    A.full = s->full ? 1 : 0;
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
    A.hfilter = s->d.hfilter;
    A.hfbits = s->d.hfbits;
    A.bidx = s->lookup == kLkBlocks ? s->d.bidx : nullptr;
    A.bstart = s->lookup == kLkBlocks ? s->d.bstart : nullptr;
    A.aidx = s->lookup == kLkBlocks ? s->d.aidx : nullptr;
    A.astart = s->lookup == kLkBlocks ? s->d.astart : nullptr;
    A.arow = s->lookup == kLkBlocks ? s->d.arow : nullptr;
    A.abeta = s->lookup == kLkBlocks ? s->d.abeta : nullptr;
    A.hptr = s->ham_kernel == 4 ? s->d.hptr : nullptr;
    A.hcol = s->ham_kernel == 4 ? s->d.hcol : nullptr;
    A.hval = s->ham_kernel == 4 ? s->d.hval : nullptr;
    A.hcb = s->d.hcb;
    A.hcs = s->d.hcs;
    const bool sl = s->ham_kernel == 4 && s->d.scb > 0;
    A.sbase = sl ? s->d.sbase : nullptr;
    A.sgbase = sl ? s->d.sgbase : nullptr;
    A.sglen = sl ? s->d.sglen : nullptr;
    A.sperm = sl ? s->d.sperm : nullptr;
    A.scol = sl ? s->d.scol : nullptr;
    A.sval = sl ? s->d.sval : nullptr;
    A.spart = sl ? s->d.spart : nullptr;
    A.scb = s->d.scb;
    A.scs = s->d.scs;
    A.sgroups = s->d.sgroups;
    A.rankA = s->d.rankA;
    A.rankB = s->d.rankB;
    return A;
}

static hipError_t launch_ham_product(const irl_system *s, const double *w, double *u, int64_t b0, int64_t b1,
                                     hipStream_t st);

int64_t ham_row_quantum(const irl_system *s) { return s->ham_kernel == 2 ? s->nA : 1; }

hipError_t launch_ham_apply_rows(const irl_system *s, const double *w, double *u, int64_t r0, int64_t r1,
                                 hipStream_t st)
{
    if (r0 < 0 || r1 > s->ns || r0 > r1) return hipErrorInvalidValue;
    if (r0 == r1) return hipSuccess;
    if (s->ham_kernel == 2) {
        // the string-product kernel works on whole beta strings
        if (r0 % s->nA || r1 % s->nA) return hipErrorInvalidValue;
        return launch_ham_product(s, w, u, r0 / s->nA, r1 / s->nA, st);
    }
    HamArgs A = ham_view(s);
    int64_t blocks = (r1 - r0 + 3) / 4;
    // the enumerating kernels take rows in grid strides and sum each row on one
    // wavefront, so the cap and the wavefronts per workgroup (both tunable) only move
    // rows between workgroups.  By default every group of rows gets its own workgroup
    // up to 2^20 of them (c3: 72.7 ms per apply against 83.7 ms with a cap of 65,536
    // and four groups per workgroup: the rows' costs vary, and the hardware's dispatch
    // of waiting workgroups balances them better than a fixed stride does)
    const int64_t cap = s->ham_kernel == 4 ? 65536 : (s->tune_pull_blocks > 0 ? s->tune_pull_blocks : (1 << 20));
    if (blocks > cap) blocks = cap;
    if (s->ham_kernel == 4 && A.sval) return launch_ham_sliced(s, A, w, u, r0, r1, st);
    if (s->ham_kernel == 4) {
        for (int b = 0; b < A.hcb; ++b) {
            k_ham_stored<<<(unsigned)blocks, 256, 0, st>>>(A, w, u, r0, r1, b);
            const hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    }
    // wavefronts (rows) per workgroup of the enumerating kernels (tunable; one row
    // per wavefront whatever the count).  Default: one with the small lists (c3:
    // 57.2 ms against 59.3 with four), four with the large ones
    const int nw = s->tune_pull_waves > 0 ? s->tune_pull_waves : (s->n <= kSmallListsMaxN ? 1 : 4);
    if (s->lookup == kLkBlocks)
        launch_pull<kLkBlocks>(A, w, u, r0, r1, nw, cap, st);
    else if (s->lookup == kLkHash)
        launch_pull<kLkHash>(A, w, u, r0, r1, nw, cap, st);
    else
        launch_pull<kLkRanks>(A, w, u, r0, r1, nw, cap, st);
    return hipGetLastError();
}

hipError_t launch_ham_apply(const irl_system *s, const double *w, double *u, hipStream_t st)
{
    return launch_ham_apply_rows(s, w, u, 0, s->ns, st);
}

hipError_t launch_ham_count(const irl_system *s, int32_t *count, hipStream_t st)
{
    HamArgs A = ham_view(s);
    int64_t blocks = (s->ns + 3) / 4;
    if (blocks > 65536) blocks = 65536;
    if (s->lookup == kLkBlocks)
        k_ham_count<kLkBlocks><<<(unsigned)blocks, 256, 0, st>>>(A, count);
    else if (s->lookup == kLkHash)
        k_ham_count<kLkHash><<<(unsigned)blocks, 256, 0, st>>>(A, count);
    else
        k_ham_count<kLkRanks><<<(unsigned)blocks, 256, 0, st>>>(A, count);
    return hipGetLastError();
}

hipError_t launch_ham_fill(const irl_system *s, const int64_t *ptr, int32_t *col, double *val,
                           hipStream_t st)
{
    HamArgs A = ham_view(s);
    int64_t blocks = (s->ns + 3) / 4;
    if (blocks > 65536) blocks = 65536;
    if (s->lookup == kLkBlocks)
        k_ham_fill<kLkBlocks><<<(unsigned)blocks, 256, 0, st>>>(A, ptr, col, val);
    else if (s->lookup == kLkHash)
        k_ham_fill<kLkHash><<<(unsigned)blocks, 256, 0, st>>>(A, ptr, col, val);
    else
        k_ham_fill<kLkRanks><<<(unsigned)blocks, 256, 0, st>>>(A, ptr, col, val);
    return hipGetLastError();
}

// Connections of one row (debug surface): same candidate enumeration as the
// apply kernel, one lane, written in enumeration order.
template <int LK>
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
    if constexpr (LK == kLkBlocks) {
        build_block_ranges(A, L, al, be, lane);
        __syncthreads();
    }
    if (lane != 0) return;
    int c = 0;
    visit_row<LK>(A, L, al, be, 0, 1, [&](int64_t r, int sg, int k, double v) {
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
    HamArgs A = ham_view(s);
    if (s->lookup == kLkBlocks)
        k_ham_row_list<kLkBlocks><<<1, 64, 0, st>>>(A, row, tgt, sign, kind, val, count, cap);
    else if (s->lookup == kLkHash)
        k_ham_row_list<kLkHash><<<1, 64, 0, st>>>(A, row, tgt, sign, kind, val, count, cap);
    else
        k_ham_row_list<kLkRanks><<<1, 64, 0, st>>>(A, row, tgt, sign, kind, val, count, cap);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// String-product kernel for a full (N_alpha, N_beta) space.
//
// Rows with the same beta string are contiguous (row = rank(beta) * nA +
// rank(alpha)).  Per-string tables hold, for every alpha (beta) string, its
// single moves (target rank, fermionic sign, orbitals), the same-spin part of
// each single's matrix element, its same-spin double moves with their signed
// elements, and J[pq] = sum_{j in string} (pq|jj).  One workgroup takes one
// beta string and 256 alpha strings (one thread per determinant):
//   alpha singles / alpha-alpha doubles gather w inside the beta row (L1),
//   beta singles / beta-beta doubles read w coalesced across the threads,
//   opposite-spin doubles loop over the beta moves (uniform) with the g slice
//   (. . | j b) in LDS and the thread's alpha moves cached in registers.
// The elements are the same Slater-Condon expressions as above, summed in a
// different (fixed) order.
// ---------------------------------------------------------------------------
constexpr int kProdThreads = 256;
constexpr int kProdMaxSingles = 64;     // n_e * (n - n_e) per spin
constexpr int kProdMaxDoubles = 1024;   // C(n_e, 2) C(n - n_e, 2) per spin

struct StrTables {
    int32_t *srank;   // [e][s]  target rank
    uint16_t *sia;    // [e][s]  i | a << 5 | (sign < 0) << 10
    double *sf;       // [e][s]  h_ia + sum_{j in s}[(ia|jj) - (ij|ja)]
    int32_t *drank;   // [d][s]
    double *dval;     // [d][s]  signed element
    double *J;        // [pq][s] sum_{j in s} (pq|jj)
};

__global__ void k_string_tables(const uint32_t *strs, const int32_t *rank, int64_t nstr, int n,
                                int ne, const double *h, const double *g, StrTables T)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nstr) return;
    const uint32_t bits = strs[s];
    const uint32_t full = (n == 32) ? 0xffffffffu : ((1u << n) - 1u);
    const uint32_t vir = ~bits & full;
    int e = 0;
    for (uint32_t bi = bits; bi; bi &= bi - 1) {
        const int i = __ffs(bi) - 1;
        for (uint32_t ba = vir; ba; ba &= ba - 1) {
            const int a = __ffs(ba) - 1;
            const int sg = move_sign(bits, i, a);
            const uint32_t nb = (bits & ~(1u << i)) | (1u << a);
            double f = h[i * n + a];
            for (uint32_t bj = bits; bj; bj &= bj - 1) {
                const int j = __ffs(bj) - 1;
                f += gint(g, n, i, a, j, j) - gint(g, n, i, j, j, a);
            }
            T.srank[(int64_t)e * nstr + s] = rank[nb];
            T.sia[(int64_t)e * nstr + s] = (uint16_t)(i | (a << 5) | ((sg < 0 ? 1 : 0) << 10));
            T.sf[(int64_t)e * nstr + s] = f;
            ++e;
        }
    }
    int d = 0;
    for (uint32_t bi = bits; bi; bi &= bi - 1) {
        const int i = __ffs(bi) - 1;
        for (uint32_t bj = bi & (bi - 1); bj; bj &= bj - 1) {
            const int j = __ffs(bj) - 1;
            for (uint32_t ba = vir; ba; ba &= ba - 1) {
                const int a = __ffs(ba) - 1;
                for (uint32_t bb = ba & (ba - 1); bb; bb &= bb - 1) {
                    const int b = __ffs(bb) - 1;
                    const int s1 = move_sign(bits, i, a);
                    const uint32_t b1 = (bits & ~(1u << i)) | (1u << a);
                    const int s2 = move_sign(b1, j, b);
                    const uint32_t b2 = (b1 & ~(1u << j)) | (1u << b);
                    T.drank[(int64_t)d * nstr + s] = rank[b2];
                    T.dval[(int64_t)d * nstr + s] =
                        (s1 * s2) * (gint(g, n, i, a, j, b) - gint(g, n, i, b, j, a));
                    ++d;
                }
            }
        }
    }
    for (int p = 0; p < n; ++p)
        for (int q = 0; q < n; ++q) {
            double acc = 0.0;
            for (uint32_t bj = bits; bj; bj &= bj - 1) {
                const int j = __ffs(bj) - 1;
                acc += gint(g, n, p, q, j, j);
            }
            T.J[(int64_t)(p * n + q) * nstr + s] = acc;
        }
}

struct ProdArgs {
    int n, nsa, nsb, nda, ndb;
    int64_t nA, nB;
    int64_t rb0;              // first beta string of the launch (blockIdx.y + rb0)
    int dense;                // same-spin doubles applied by dense products instead
    const double *diag, *g;
    StrTables A, B;
};

template <int NSA>
__global__ __launch_bounds__(kProdThreads) void k_ham_product(ProdArgs P, const double *__restrict__ w,
                                                              double *__restrict__ u)
{
    __shared__ double gs[32 * 32];          // (p q | j_f b_f) for all p, q
    __shared__ double jb[32 * 32];          // sum_{j in beta} (pq|jj)
    __shared__ int32_t sb_rank[kProdMaxSingles];
    __shared__ uint16_t sb_ia[kProdMaxSingles];
    __shared__ double sb_f[kProdMaxSingles];
    __shared__ int32_t db_rank[kProdMaxDoubles];
    __shared__ double db_val[kProdMaxDoubles];
    const int n = P.n, n2 = n * n;
    const int64_t rb = blockIdx.y + P.rb0;
    const int64_t ra = (int64_t)blockIdx.x * kProdThreads + threadIdx.x;
    const bool valid = ra < P.nA;
    const int64_t rac = valid ? ra : 0;
    for (int p = threadIdx.x; p < n2; p += kProdThreads) jb[p] = P.B.J[(int64_t)p * P.nB + rb];
    for (int f = threadIdx.x; f < P.nsb; f += kProdThreads) {
        sb_rank[f] = P.B.srank[(int64_t)f * P.nB + rb];
        sb_ia[f] = P.B.sia[(int64_t)f * P.nB + rb];
        sb_f[f] = P.B.sf[(int64_t)f * P.nB + rb];
    }
    for (int d = threadIdx.x; d < P.ndb; d += kProdThreads) {
        db_rank[d] = P.B.drank[(int64_t)d * P.nB + rb];
        db_val[d] = P.B.dval[(int64_t)d * P.nB + rb];
    }
    __syncthreads();
    const double *wrow = w + rb * P.nA;
    double acc = P.diag[rb * P.nA + rac] * wrow[rac];
    // alpha singles (moves cached in registers for the opposite-spin loop)
    int32_t ar[NSA];
    uint16_t aia[NSA];
#pragma unroll
    for (int e = 0; e < NSA; ++e) {
        if (e < P.nsa) {
            ar[e] = P.A.srank[(int64_t)e * P.nA + rac];
            aia[e] = P.A.sia[(int64_t)e * P.nA + rac];
            const int i = aia[e] & 31, a = (aia[e] >> 5) & 31;
            const double v = P.A.sf[(int64_t)e * P.nA + rac] + jb[i * n + a];
            acc += ((aia[e] >> 10) & 1 ? -v : v) * wrow[ar[e]];
        } else {
            ar[e] = 0;
            aia[e] = 0;
        }
    }
    // alpha-alpha doubles
    if (!P.dense)
        for (int d = 0; d < P.nda; ++d)
            acc += P.A.dval[(int64_t)d * P.nA + rac] * wrow[P.A.drank[(int64_t)d * P.nA + rac]];
    // beta singles: opposite-spin part sum_{i in alpha} (jb|ii) from the alpha J table
    for (int f = 0; f < P.nsb; ++f) {
        const int j = sb_ia[f] & 31, b = (sb_ia[f] >> 5) & 31;
        const double v = sb_f[f] + P.A.J[(int64_t)(j * n + b) * P.nA + rac];
        acc += ((sb_ia[f] >> 10) & 1 ? -v : v) * w[(int64_t)sb_rank[f] * P.nA + rac];
    }
    // beta-beta doubles
    if (!P.dense)
        for (int d = 0; d < P.ndb; ++d) acc += db_val[d] * w[(int64_t)db_rank[d] * P.nA + rac];
    // opposite-spin doubles
    for (int f = 0; f < P.nsb; ++f) {
        const int j = sb_ia[f] & 31, b = (sb_ia[f] >> 5) & 31;
        __syncthreads();
        for (int p = threadIdx.x; p < n2; p += kProdThreads)
            gs[p] = P.g[(int64_t)p * n2 + j * n + b];
        __syncthreads();
        const double *wb = w + (int64_t)sb_rank[f] * P.nA;
        double part = 0.0;
#pragma unroll
        for (int e = 0; e < NSA; ++e) {
            if (e < P.nsa) {
                const int i = aia[e] & 31, a = (aia[e] >> 5) & 31;
                const double v = gs[i * n + a] * wb[ar[e]];
                part += (aia[e] >> 10) & 1 ? -v : v;
            }
        }
        acc += (sb_ia[f] >> 10) & 1 ? -part : part;
    }
    if (valid) u[rb * P.nA + ra] = acc;
}

// LDS-staged variant (nA <= kProdLdsMaxA): the own beta row of w, the beta' row
// of the current beta move and the g slice live in LDS.  The g slice is staged
// multiplied by the beta move's sign, followed by its negation and one zero, so
// every alpha move of a thread is two LDS byte offsets held in registers (its
// w entry; its g entry with the alpha sign chosen by the copy, moves past nsa
// pointing at the zero): an opposite-spin term is two LDS reads and one FMA,
// with no branch.  Rows of the next beta move are loaded into registers while
// the current one is summed (two barriers per move).  TPB threads per block
// (one thread per alpha string of the block's slice).
constexpr int kProd2Threads = 512;
constexpr int kProdLdsMaxA = 2048;

template <int NSA, int TPB>
__global__ __launch_bounds__(TPB) void k_ham_product_lds(ProdArgs P, const double *__restrict__ w,
                                                         double *__restrict__ u)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int n = P.n, n2 = n * n;
    const int nA = (int)P.nA;
    double *wself = reinterpret_cast<double *>(smem);
    double *wb = wself + nA;
    double *gs = wb + nA;                  // [sign_f g | -sign_f g | 0]: 2 n2 + 1
    double *jbl = gs + 2 * n2 + 1;
    double *sb_f = jbl + n2;
    double *db_val = sb_f + P.nsb;
    int32_t *sb_rank = reinterpret_cast<int32_t *>(db_val + P.ndb);
    int32_t *db_rank = sb_rank + P.nsb;
    uint16_t *sb_ia = reinterpret_cast<uint16_t *>(db_rank + P.ndb);

    const int64_t rb = blockIdx.y + P.rb0;
    const int ra = blockIdx.x * TPB + threadIdx.x;
    const bool valid = ra < nA;
    const int rac = valid ? ra : 0;
    const double *wrow = w + rb * P.nA;
    for (int p = threadIdx.x; p < nA; p += TPB) wself[p] = wrow[p];
    for (int p = threadIdx.x; p < n2; p += TPB) jbl[p] = P.B.J[(int64_t)p * P.nB + rb];
    for (int f = threadIdx.x; f < P.nsb; f += TPB) {
        sb_rank[f] = P.B.srank[(int64_t)f * P.nB + rb];
        sb_ia[f] = P.B.sia[(int64_t)f * P.nB + rb];
        sb_f[f] = P.B.sf[(int64_t)f * P.nB + rb];
    }
    for (int d = threadIdx.x; d < P.ndb; d += TPB) {
        db_rank[d] = P.B.drank[(int64_t)d * P.nB + rb];
        db_val[d] = P.B.dval[(int64_t)d * P.nB + rb];
    }
    if (threadIdx.x == 0) gs[2 * n2] = 0.0;
    __syncthreads();
    double acc = P.diag[rb * P.nA + rac] * wself[rac];
    // alpha singles; their opposite-spin operand offsets
    const uint32_t wb_off = (uint32_t)((unsigned char *)wb - smem);
    const uint32_t gs_off = (uint32_t)((unsigned char *)gs - smem);
    uint32_t ow[NSA], og[NSA];
#pragma unroll
    for (int e = 0; e < NSA; ++e) {
        if (e < P.nsa) {
            const int32_t rk = P.A.srank[(int64_t)e * P.nA + rac];
            const uint16_t q = P.A.sia[(int64_t)e * P.nA + rac];
            const int i = q & 31, a = (q >> 5) & 31, neg = (q >> 10) & 1;
            const double v = P.A.sf[(int64_t)e * P.nA + rac] + jbl[i * n + a];
            acc += (neg ? -v : v) * wself[rk];
            ow[e] = wb_off + 8u * (uint32_t)rk;
            og[e] = gs_off + 8u * (uint32_t)(i * n + a + (neg ? n2 : 0));
        } else {
            ow[e] = wb_off;
            og[e] = gs_off + 8u * (uint32_t)(2 * n2);
        }
    }
    if (!P.dense)
        for (int d = 0; d < P.nda; ++d)
            acc += P.A.dval[(int64_t)d * P.nA + rac] * wself[P.A.drank[(int64_t)d * P.nA + rac]];
    for (int f = 0; f < P.nsb; ++f) {
        const int j = sb_ia[f] & 31, b = (sb_ia[f] >> 5) & 31;
        const double v = sb_f[f] + P.A.J[(int64_t)(j * n + b) * P.nA + rac];
        acc += ((sb_ia[f] >> 10) & 1 ? -v : v) * w[(int64_t)sb_rank[f] * P.nA + rac];
    }
    if (!P.dense)
        for (int d = 0; d < P.ndb; ++d) acc += db_val[d] * w[(int64_t)db_rank[d] * P.nA + rac];

    // opposite-spin doubles
    constexpr int PFW = (kProdLdsMaxA + TPB - 1) / TPB;
    constexpr int PFG = (32 * 32 + TPB - 1) / TPB;
    double pw[PFW], pg[PFG];
    auto fetch = [&](int f) {
        const int j = sb_ia[f] & 31, b = (sb_ia[f] >> 5) & 31;
        const double *src = w + (int64_t)sb_rank[f] * P.nA;
#pragma unroll
        for (int t = 0; t < PFW; ++t) {
            const int p = threadIdx.x + t * TPB;
            pw[t] = p < nA ? src[p] : 0.0;
        }
#pragma unroll
        for (int t = 0; t < PFG; ++t) {
            const int p = threadIdx.x + t * TPB;
            pg[t] = p < n2 ? P.g[(int64_t)p * n2 + j * n + b] : 0.0;
        }
    };
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    if (P.nsb > 0) fetch(0);
    for (int f = 0; f < P.nsb; ++f) {
        const double sg = (sb_ia[f] >> 10) & 1 ? -1.0 : 1.0;
        __syncthreads();                   // every read of the previous move is done
#pragma unroll
        for (int t = 0; t < PFW; ++t) {
            const int p = threadIdx.x + t * TPB;
            if (p < nA) wb[p] = pw[t];
        }
#pragma unroll
        for (int t = 0; t < PFG; ++t) {
            const int p = threadIdx.x + t * TPB;
            if (p < n2) {
                gs[p] = sg * pg[t];
                gs[n2 + p] = -sg * pg[t];
            }
        }
        __syncthreads();
        if (f + 1 < P.nsb) fetch(f + 1);
#pragma unroll
        for (int e = 0; e < NSA; e += 4) {
            s0 = fma(*(const double *)(smem + og[e]), *(const double *)(smem + ow[e]), s0);
            if (e + 1 < NSA) s1 = fma(*(const double *)(smem + og[e + 1]), *(const double *)(smem + ow[e + 1]), s1);
            if (e + 2 < NSA) s2 = fma(*(const double *)(smem + og[e + 2]), *(const double *)(smem + ow[e + 2]), s2);
            if (e + 3 < NSA) s3 = fma(*(const double *)(smem + og[e + 3]), *(const double *)(smem + ow[e + 3]), s3);
        }
    }
    acc += (s0 + s1) + (s2 + s3);
    if (valid) u[rb * P.nA + ra] = acc;
}

static size_t product_lds_bytes(const ProdArgs &P)
{
    const size_t n2 = (size_t)P.n * P.n;
    return (2 * (size_t)P.nA + 3 * n2 + 1 + P.nsb + P.ndb) * 8 + (size_t)(P.nsb + P.ndb) * 4 +
           (size_t)P.nsb * 2;
}

static bool product_fits(const irl_system *s, int &nsa, int &nsb, int &nda, int &ndb)
{
    const int n = s->n, na = s->na, nb = s->nb, va = n - na, vb = n - nb;
    nsa = na * va;
    nsb = nb * vb;
    nda = na * (na - 1) / 2 * (va * (va - 1) / 2);
    ndb = nb * (nb - 1) / 2 * (vb * (vb - 1) / 2);
    if (!s->full || n > 20 || s->nB > 65535) return false;
    if (nsa > kProdMaxSingles || nsb > kProdMaxSingles) return false;
    if (nda > kProdMaxDoubles || ndb > kProdMaxDoubles) return false;
    const double bytes = (double)(s->nA + s->nB) * ((nsa > nsb ? nsa : nsb) * 14.0 +
                                                    (nda > ndb ? nda : ndb) * 12.0 + n * n * 8.0);
    return bytes < 4e9;
}

// Same-spin doubles of one spin as a dense symmetric matrix D[s][t] (row s = string
// rank, t = target rank): the element of string s and its double t.
__global__ void k_dense_doubles(const int32_t *__restrict__ drank, const double *__restrict__ dval, int64_t nstr,
                                int nd, double *__restrict__ D)
{
    const int64_t str = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (str >= nstr) return;
    for (int d = 0; d < nd; ++d) D[str * nstr + drank[(int64_t)d * nstr + str]] = dval[(int64_t)d * nstr + str];
}

// strings per spin up to which the same-spin doubles are dense products
constexpr int64_t kDenseDoublesMax = 2048;

void free_dense_doubles(irl_system *s)
{
    for (double **p : {&s->d.denseA, &s->d.denseB}) {
        if (*p) (void)hipFree(*p);
        *p = nullptr;
    }
}

// Dense same-spin doubles for a full space with few strings per spin: a DGEMM per
// spin replaces 2 x C(N,2) C(n-N,2) gathered terms per determinant.
static hipError_t build_dense_doubles(irl_system *s, int nda, int ndb, hipStream_t st)
{
    if (s->nA > kDenseDoublesMax || s->nB > kDenseDoublesMax) return hipSuccess;
    hipError_t e;
    const size_t bA = (size_t)s->nA * s->nA * 8, bB = (size_t)s->nB * s->nB * 8;
    if ((e = hipMalloc(&s->d.denseA, bA)) != hipSuccess) return e;
    if ((e = hipMalloc(&s->d.denseB, bB)) != hipSuccess) return e;
    s->dev_bytes += bA + bB;
    if ((e = hipMemsetAsync(s->d.denseA, 0, bA, st)) != hipSuccess) return e;
    if ((e = hipMemsetAsync(s->d.denseB, 0, bB, st)) != hipSuccess) return e;
    k_dense_doubles<<<(unsigned)((s->nA + 127) / 128), 128, 0, st>>>(s->d.dblA_rank, s->d.dblA_val, s->nA, nda,
                                                                     s->d.denseA);
    k_dense_doubles<<<(unsigned)((s->nB + 127) / 128), 128, 0, st>>>(s->d.dblB_rank, s->d.dblB_val, s->nB, ndb,
                                                                     s->d.denseB);
    return hipGetLastError();
}

// ---- same-spin doubles as one FP64 matrix-core product ------------------------
// With w as the column-major nA x nB matrix X (column = beta string) and D_A, D_B
// the symmetric same-spin double matrices of each spin,
//     U[:, b0:b1] += D_A X[:, b0:b1] + X D_B[:, b0:b1].
// A workgroup owns a 64 x 64 tile of U and has two groups of 4 wavefronts: group 0
// forms the tile of D_A X, group 1 that of X D_B, each wavefront a 32 x 32 quarter
// as 2 x 2 blocks of v_mfma_f64_16x16x4f64, over inner tiles of 32 staged through
// its own double-buffered LDS (the next inner tile is loaded while the current one
// is multiplied; two groups per workgroup put two wavefronts on every SIMD).  At
// the end group 1 hands its tile to group 0 through LDS, which adds the two in a
// fixed order and updates U once.  Operand layout of the instruction (lane l):
// A[l % 16][l / 16], B[l / 16][l % 16]; result register r holds D[4 r + l / 16][l % 16].
namespace {
constexpr int kDblTM = 64, kDblTN = 64, kDblTK = 32, kDblThreads = 512;
constexpr int kDblLdB = kDblTN + 1;   // padded rows of the B tile (conflict-free column stores)
constexpr int kDblPer = kDblTM * kDblTK / 256;   // tile elements per thread of a group (8)

typedef double dbl4 __attribute__((ext_vector_type(4)));

struct DblArgs {
    const double *DA, *DB, *X;   // nA x nA, nB x nB, nA x nB (column-major)
    double *U;                   // nA x nB, columns [b0, b1) updated
    int64_t nA, nB, b0, nbeta;
};

struct DblRegs {
    double a[kDblPer], b[kDblPer];
    uint32_t va, vb;   // bit j: element j is inside the matrices (else it enters as zero)
};

struct DblTiles {
    double A[2][kDblTK][kDblTM];
    double B[2][kDblTK][kDblLdB];
};
}  // namespace

__global__ void __launch_bounds__(kDblThreads) k_same_spin_doubles(DblArgs a)
{
    __shared__ DblTiles tiles[2];
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6, grp = wv >> 2, wq = wv & 3, tg = t & 255;
    DblTiles &T = tiles[grp];
    const int64_t m0 = (int64_t)blockIdx.x * kDblTM, n0 = (int64_t)blockIdx.y * kDblTN;
    const int64_t M = a.nA, N = a.nbeta;
    // group 0: A = D_A (ld nA), B = X[:, b0 + n] (ld nA), inner index over nA;
    // group 1: A = X (ld nA), B = D_B[:, b0 + n] (ld nB), inner index over nB
    const double *Am = grp ? a.X : a.DA;
    const double *Bm = grp ? a.DB : a.X;
    const int64_t K = grp ? a.nB : a.nA;
    const int64_t ldb = grp ? a.nB : a.nA;
    const int nkt = (int)((K + kDblTK - 1) / kDblTK);
    const int nkmax = (int)((((a.nA > a.nB) ? a.nA : a.nB) + kDblTK - 1) / kDblTK);
    // A tile element (row m0 + tg % 64, inner k0 + tg / 64 + 4 j); B tile element
    // (inner k0 + tg % 32, column n0 + tg / 32 + 8 j).  Out-of-range elements load a
    // clamped in-range address and enter as zero (masks applied at the LDS store).
    const int ar = tg & 63, ak = tg >> 6, bk = tg & 31, bn = tg >> 5;
    auto load = [&](int kt, DblRegs &R) {
        const int64_t k0 = (int64_t)kt * kDblTK;
        const int64_t m = m0 + ar, mc = m < M ? m : M - 1;
        R.va = R.vb = 0u;
#pragma unroll
        for (int j = 0; j < kDblPer; ++j) {
            const int64_t k = k0 + ak + 4 * j, kc = k < K ? k : K - 1;
            R.a[j] = Am[kc * a.nA + mc];
            R.va |= (m < M && k < K) ? (1u << j) : 0u;
        }
        const int64_t kb = k0 + bk, kbc = kb < K ? kb : K - 1;
#pragma unroll
        for (int j = 0; j < kDblPer; ++j) {
            const int64_t n = n0 + bn + 8 * j, nc = n < N ? n : N - 1;
            R.b[j] = Bm[(a.b0 + nc) * ldb + kbc];
            R.vb |= (n < N && kb < K) ? (1u << j) : 0u;
        }
    };
    auto store = [&](int buf, const DblRegs &R) {
#pragma unroll
        for (int j = 0; j < kDblPer; ++j) T.A[buf][ak + 4 * j][ar] = ((R.va >> j) & 1u) ? R.a[j] : 0.0;
#pragma unroll
        for (int j = 0; j < kDblPer; ++j) T.B[buf][bk][bn + 8 * j] = ((R.vb >> j) & 1u) ? R.b[j] : 0.0;
    };
    dbl4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = dbl4{0.0, 0.0, 0.0, 0.0};
    const int wm = (wq & 1) * 32, wn = (wq >> 1) * 32;
    const int lr = lane & 15, lk = lane >> 4;
    auto compute = [&](int buf) {
        double fa[2][2], fb[2][2];
#pragma unroll
        for (int i = 0; i < 2; ++i) fa[0][i] = T.A[buf][lk][wm + 16 * i + lr];
#pragma unroll
        for (int j = 0; j < 2; ++j) fb[0][j] = T.B[buf][lk][wn + 16 * j + lr];
#pragma unroll
        for (int ks = 0; ks < kDblTK; ks += 4) {
            const int c = (ks >> 2) & 1, nx = c ^ 1;
            if (ks + 4 < kDblTK) {
#pragma unroll
                for (int i = 0; i < 2; ++i) fa[nx][i] = T.A[buf][ks + 4 + lk][wm + 16 * i + lr];
#pragma unroll
                for (int j = 0; j < 2; ++j) fb[nx][j] = T.B[buf][ks + 4 + lk][wn + 16 * j + lr];
            }
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[c][i], fb[c][j], acc[i][j], 0, 0, 0);
        }
    };
    DblRegs R;
    if (nkt > 0) {
        load(0, R);
        store(0, R);
    }
    __syncthreads();
    for (int kt = 0; kt < nkmax; ++kt) {   // every wavefront meets every barrier
        const int buf = kt & 1;
        const bool more = kt + 1 < nkt;
        if (more) load(kt + 1, R);
        if (kt < nkt) compute(buf);
        if (more) store(buf ^ 1, R);
        __syncthreads();
    }
    // group 1 hands its tile to group 0 (the LDS of the inner tiles is free now)
    double *xfer = &tiles[0].A[0][0][0];
    if (grp == 1) {
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j)
#pragma unroll
                for (int r = 0; r < 4; ++r) xfer[((wq * 4 + i * 2 + j) * 4 + r) * 64 + lane] = acc[i][j][r];
    }
    __syncthreads();
    if (grp == 1) return;
    // U tile += acc_0 + acc_1 (row m0 + wm + 16 i + 4 r + l / 16, column n0 + wn + 16 j + l % 16)
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int64_t n = n0 + wn + 16 * j + lr;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t m = m0 + wm + 16 * i + 4 * r + lk;
                const double v = acc[i][j][r] + xfer[((wq * 4 + i * 2 + j) * 4 + r) * 64 + lane];
                if (n < N && m < M) a.U[(a.b0 + n) * a.nA + m] += v;
            }
        }
}

static hipError_t launch_same_spin_doubles(const irl_system *s, const double *w, double *u, int64_t b0,
                                           int64_t nbeta, hipStream_t st)
{
    if (nbeta <= 0) return hipSuccess;
    DblArgs a{s->d.denseA, s->d.denseB, w, u, s->nA, s->nB, b0, nbeta};
    dim3 grid((unsigned)((s->nA + kDblTM - 1) / kDblTM), (unsigned)((nbeta + kDblTN - 1) / kDblTN));
    k_same_spin_doubles<<<grid, kDblThreads, 0, st>>>(a);
    return hipGetLastError();
}

hipError_t launch_product_tables(irl_system *s, hipStream_t st)
{
    int nsa, nsb, nda, ndb;
    if (s->ham_kernel != 1 || !product_fits(s, nsa, nsb, nda, ndb)) return hipSuccess;
    const int n = s->n;
    auto alloc = [&](StrTables &T, int64_t nstr, int ns1, int nd) -> hipError_t {
        hipError_t e;
        if ((e = hipMalloc(&T.srank, (size_t)(ns1 ? ns1 : 1) * nstr * 4)) != hipSuccess) return e;
        if ((e = hipMalloc(&T.sia, (size_t)(ns1 ? ns1 : 1) * nstr * 2)) != hipSuccess) return e;
        if ((e = hipMalloc(&T.sf, (size_t)(ns1 ? ns1 : 1) * nstr * 8)) != hipSuccess) return e;
        if ((e = hipMalloc(&T.drank, (size_t)(nd ? nd : 1) * nstr * 4)) != hipSuccess) return e;
        if ((e = hipMalloc(&T.dval, (size_t)(nd ? nd : 1) * nstr * 8)) != hipSuccess) return e;
        if ((e = hipMalloc(&T.J, (size_t)n * n * nstr * 8)) != hipSuccess) return e;
        s->dev_bytes += (size_t)nstr * ((ns1 ? ns1 : 1) * 14 + (nd ? nd : 1) * 12 + n * n * 8);
        return hipSuccess;
    };
    StrTables A{}, B{};
    hipError_t e;
    if ((e = alloc(A, s->nA, nsa, nda)) != hipSuccess) return e;
    s->d.sglA = reinterpret_cast<uint32_t *>(A.srank);
    s->d.sglA_ia = A.sia;
    s->d.fA = A.sf;
    s->d.dblA_rank = A.drank;
    s->d.dblA_val = A.dval;
    s->d.jA = A.J;
    if ((e = alloc(B, s->nB, nsb, ndb)) != hipSuccess) return e;
    s->d.sglB = reinterpret_cast<uint32_t *>(B.srank);
    s->d.sglB_ia = B.sia;
    s->d.fB = B.sf;
    s->d.dblB_rank = B.drank;
    s->d.dblB_val = B.dval;
    s->d.jB = B.J;
    k_string_tables<<<(unsigned)((s->nA + 127) / 128), 128, 0, st>>>(s->d.strA, s->d.rankA, s->nA, n,
                                                                    s->na, s->d.h, s->d.g, A);
    k_string_tables<<<(unsigned)((s->nB + 127) / 128), 128, 0, st>>>(s->d.strB, s->d.rankB, s->nB, n,
                                                                    s->nb, s->d.h, s->d.g, B);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = build_dense_doubles(s, nda, ndb, st)) != hipSuccess) return e;
    s->ham_kernel = 2;
    return hipSuccess;
}

static StrTables tables_of(const irl_system *s, bool alpha)
{
    StrTables T;
    T.srank = reinterpret_cast<int32_t *>(alpha ? s->d.sglA : s->d.sglB);
    T.sia = alpha ? s->d.sglA_ia : s->d.sglB_ia;
    T.sf = alpha ? s->d.fA : s->d.fB;
    T.drank = alpha ? s->d.dblA_rank : s->d.dblB_rank;
    T.dval = alpha ? s->d.dblA_val : s->d.dblB_val;
    T.J = alpha ? s->d.jA : s->d.jB;
    return T;
}

template <int NSA>
static void launch_prod_inst(const ProdArgs &P, int64_t nbeta, const double *w, double *u, hipStream_t st)
{
    const size_t lds = product_lds_bytes(P);
    if (P.nA <= kProdLdsMaxA && lds <= 64 * 1024) {
        dim3 grid((unsigned)((P.nA + kProd2Threads - 1) / kProd2Threads), (unsigned)nbeta);
        k_ham_product_lds<NSA, kProd2Threads><<<grid, kProd2Threads, lds, st>>>(P, w, u);
    } else {
        dim3 grid((unsigned)((P.nA + kProdThreads - 1) / kProdThreads), (unsigned)nbeta);
        k_ham_product<NSA><<<grid, kProdThreads, 0, st>>>(P, w, u);
    }
}

// beta strings [b0, b1)
static hipError_t launch_ham_product(const irl_system *s, const double *w, double *u, int64_t b0, int64_t b1,
                                     hipStream_t st)
{
    ProdArgs P;
    P.rb0 = b0;
    P.dense = s->d.denseA != nullptr && s->d.denseB != nullptr;
    const int64_t nbeta = b1 - b0;
    product_fits(s, P.nsa, P.nsb, P.nda, P.ndb);
    P.n = s->n;
    P.nA = s->nA;
    P.nB = s->nB;
    P.diag = s->d.diag;
    P.g = s->d.g;
    P.A = tables_of(s, true);
    P.B = tables_of(s, false);
    const int q = (P.nsa + 3) / 4;
    switch (q) {
    case 0: case 1: launch_prod_inst<4>(P, nbeta, w, u, st); break;
    case 2: launch_prod_inst<8>(P, nbeta, w, u, st); break;
    case 3: launch_prod_inst<12>(P, nbeta, w, u, st); break;
    case 4: launch_prod_inst<16>(P, nbeta, w, u, st); break;
    case 5: launch_prod_inst<20>(P, nbeta, w, u, st); break;
    case 6: launch_prod_inst<24>(P, nbeta, w, u, st); break;
    case 7: launch_prod_inst<28>(P, nbeta, w, u, st); break;
    case 8: launch_prod_inst<32>(P, nbeta, w, u, st); break;
    case 9: launch_prod_inst<36>(P, nbeta, w, u, st); break;
    case 10: launch_prod_inst<40>(P, nbeta, w, u, st); break;
    case 11: launch_prod_inst<44>(P, nbeta, w, u, st); break;
    case 12: launch_prod_inst<48>(P, nbeta, w, u, st); break;
    case 13: launch_prod_inst<52>(P, nbeta, w, u, st); break;
    case 14: launch_prod_inst<56>(P, nbeta, w, u, st); break;
    case 15: launch_prod_inst<60>(P, nbeta, w, u, st); break;
    default: launch_prod_inst<64>(P, nbeta, w, u, st); break;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !P.dense) return e;
    return launch_same_spin_doubles(s, w, u, b0, nbeta, st);
}

}  // namespace irl
