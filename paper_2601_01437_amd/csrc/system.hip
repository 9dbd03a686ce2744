// Determinant set, key -> row lookup and Hamiltonian diagonal on gfx950.
//
// Determinant space (Methods, "Wave Function Ansatz"; particle-number
// constraint of Eq. constraint): all alpha strings with n_alpha bits times all
// beta strings with n_beta bits, or a caller-supplied subset.  Keys ascend
// (beta string major), so row r of a full space is rank(beta) * nA + rank(alpha),
// where the rank of a string is its position in ascending integer order
// (combinatorial number system: rank = sum_t C(c_t, t) over its set bits
// c_1 < c_2 < ... , t = 1, 2, ...).
#include <mutex>

#include "internal.h"

namespace irl {

__device__ __forceinline__ uint64_t mix64(uint64_t x)
{
    // MurmurHash3 64-bit finaliser
    x ^= x >> 33;
    x *= 0xff51afd7ed558ccdull;
    x ^= x >> 33;
    x *= 0xc4ceb9fe1a85ec53ull;
    x ^= x >> 33;
    return x;
}

__device__ __forceinline__ int64_t binom(int c, int t)
{
    if (t < 0 || c < t) return 0;
    int64_t r = 1;
    for (int i = 1; i <= t; ++i) r = r * (c - t + i) / i;   // exact at every step
    return r;
}

// rank table over all 2^n strings, plus the inverse (string by rank)
__global__ void k_rank_table(int32_t *rank, uint32_t *str, int n, int ne)
{
    uint32_t bits = blockIdx.x * blockDim.x + threadIdx.x;
    if (bits >= (1u << n)) return;
    if (__popc(bits) != ne) { rank[bits] = -1; return; }
    int64_t r = 0;
    int t = 0;
    uint32_t b = bits;
    while (b) {
        int c = __ffs(b) - 1;
        b &= b - 1;
        ++t;
        r += binom(c, t);
    }
    rank[bits] = (int32_t)r;
    str[r] = bits;
}

__global__ void k_full_keys(uint64_t *keys, const uint32_t *strA, const uint32_t *strB,
                            int64_t nA, int64_t ns)
{
    int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= ns) return;
    int64_t rb = r / nA, ra = r - rb * nA;
    keys[r] = (uint64_t)strA[ra] | ((uint64_t)strB[rb] << 32);
}

hipError_t launch_enumerate_full(uint64_t *keys, uint32_t *strA, uint32_t *strB, int32_t *rankA,
                                 int32_t *rankB, int n, int na, int nb, int64_t nA, int64_t nB,
                                 hipStream_t st)
{
    const int bs = 256;
    unsigned grid = (unsigned)(((1u << n) + bs - 1) / bs);
    k_rank_table<<<grid, bs, 0, st>>>(rankA, strA, n, na);
    k_rank_table<<<grid, bs, 0, st>>>(rankB, strB, n, nb);
    int64_t ns = nA * nB;
    k_full_keys<<<(unsigned)((ns + bs - 1) / bs), bs, 0, st>>>(keys, strA, strB, nA, ns);
    return hipGetLastError();
}

__global__ void k_fill_u64(uint64_t *p, uint64_t n, uint64_t v)
{
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_hash_insert(const uint64_t *keys, int64_t ns, uint64_t *hkeys, int32_t *hrows,
                              uint64_t mask, uint32_t *filter, int fbits)
{
    int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= ns) return;
    uint64_t key = keys[r];
    const uint64_t hm = mix64(key);
    if (filter) {
        const uint64_t bit = hm >> (64 - fbits);
        atomicOr(&filter[bit >> 5], 1u << (bit & 31));
    }
    uint64_t slot = hm & mask;
    for (uint64_t probe = 0; probe <= mask; ++probe) {
        unsigned long long prev = atomicCAS((unsigned long long *)&hkeys[slot],
                                            (unsigned long long)kEmptyKey,
                                            (unsigned long long)key);
        if (prev == kEmptyKey || prev == key) {
            hrows[slot] = (int32_t)r;
            return;
        }
        slot = (slot + 1) & mask;
    }
}

__global__ void k_fill_u32(uint32_t *p, uint64_t n, uint32_t v)
{
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

hipError_t launch_hash_build(const uint64_t *keys, int64_t ns, uint64_t *hkeys, int32_t *hrows,
                             uint64_t cap, uint32_t *filter, int fbits, hipStream_t st)
{
    const int bs = 256;
    k_fill_u64<<<(unsigned)((cap + bs - 1) / bs), bs, 0, st>>>(hkeys, cap, kEmptyKey);
    if (filter) {
        const uint64_t words = (1ull << fbits) / 32;
        k_fill_u32<<<(unsigned)((words + bs - 1) / bs), bs, 0, st>>>(filter, words, 0u);
    }
    k_hash_insert<<<(unsigned)((ns + bs - 1) / bs), bs, 0, st>>>(keys, ns, hkeys, hrows, cap - 1,
                                                                filter, fbits);
    return hipGetLastError();
}

__device__ __forceinline__ int32_t hash_find(const uint64_t *hkeys, const int32_t *hrows,
                                             uint64_t mask, uint64_t key)
{
    if (key == kEmptyKey) return -1;   // the empty-slot marker is never a member
    uint64_t slot = mix64(key) & mask;
    for (uint64_t probe = 0; probe <= mask; ++probe) {
        uint64_t k = hkeys[slot];
        if (k == key) return hrows[slot];
        if (k == kEmptyKey) return -1;
        slot = (slot + 1) & mask;
    }
    return -1;
}

__global__ void k_hash_lookup(const uint64_t *hkeys, const int32_t *hrows, uint64_t mask,
                              const uint64_t *q, int64_t nq, int32_t *rows)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nq) rows[i] = hash_find(hkeys, hrows, mask, q[i]);
}

hipError_t launch_hash_lookup(const uint64_t *hkeys, const int32_t *hrows, uint64_t cap,
                              const uint64_t *q, int64_t nq, int32_t *rows, hipStream_t st)
{
    if (nq == 0) return hipSuccess;
    const int bs = 256;
    k_hash_lookup<<<(unsigned)((nq + bs - 1) / bs), bs, 0, st>>>(hkeys, hrows, cap - 1, q, nq, rows);
    return hipGetLastError();
}

// H_xx = sum_i h_ii + 1/2 sum_{i,j same spin} [(ii|jj) - (ij|ji)] + sum_{i alpha, j beta} (ii|jj)
__global__ void k_diagonal(const uint64_t *keys, int64_t ns, int n, const double *h,
                           const double *g, double *diag)
{
    int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= ns) return;
    uint64_t key = keys[r];
    uint32_t al = (uint32_t)key, be = (uint32_t)(key >> 32);
    const size_t n2 = (size_t)n * n, n3 = n2 * n;
    double e = 0.0;
    for (int spin = 0; spin < 2; ++spin) {
        uint32_t s = spin ? be : al;
        for (uint32_t bi = s; bi; bi &= bi - 1) {
            int i = __ffs(bi) - 1;
            e += h[i * n + i];
            for (uint32_t bj = s; bj; bj &= bj - 1) {
                int j = __ffs(bj) - 1;
                e += 0.5 * (g[i * n3 + i * n2 + j * n + j] - g[i * n3 + j * n2 + j * n + i]);
            }
        }
    }
    for (uint32_t bi = al; bi; bi &= bi - 1) {
        int i = __ffs(bi) - 1;
        for (uint32_t bj = be; bj; bj &= bj - 1) {
            int j = __ffs(bj) - 1;
            e += g[i * n3 + i * n2 + j * n + j];
        }
    }
    diag[r] = e;
}

hipError_t launch_diagonal(const uint64_t *keys, int64_t ns, int n, const double *h,
                           const double *g, double *diag, hipStream_t st)
{
    const int bs = 256;
    k_diagonal<<<(unsigned)((ns + bs - 1) / bs), bs, 0, st>>>(keys, ns, n, h, g, diag);
    return hipGetLastError();
}

// key -> row for any set: hash when built, else full-space string ranks
__global__ void k_lookup_ranks(const int32_t *rankA, const int32_t *rankB, int n, int64_t nA,
                               const uint64_t *q, int64_t nq, int32_t *rows)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nq) return;
    uint64_t key = q[i];
    uint32_t al = (uint32_t)key, be = (uint32_t)(key >> 32);
    if (n < 32 && ((al >> n) || (be >> n))) { rows[i] = -1; return; }
    int32_t ra = rankA[al], rb = rankB[be];
    rows[i] = (ra < 0 || rb < 0) ? -1 : (int32_t)((int64_t)rb * nA + ra);
}

hipError_t launch_lookup_any(const irl_system *s, const uint64_t *q, int64_t nq, int32_t *rows,
                             hipStream_t st)
{
    if (nq == 0) return hipSuccess;
    if (s->d.hkeys) return launch_hash_lookup(s->d.hkeys, s->d.hrows, s->d.hcap, q, nq, rows, st);
    const int bs = 256;
    k_lookup_ranks<<<(unsigned)((nq + bs - 1) / bs), bs, 0, st>>>(s->d.rankA, s->d.rankB, s->n,
                                                                  s->nA, q, nq, rows);
    return hipGetLastError();
}

// ---- fixed device scratch for callers that cannot allocate --------------------
// One array per GPU (each device that loads the library holds its own copy at its
// own address until the process ends).  Host code never passes the array's name
// to a kernel or a copy: it uses the device address resolved by
// hipGetSymbolAddress, once per device, in noalloc_scratch_setup().
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t noalloc_scratch_setup(int device)
{
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[device]) return hipSuccess;
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device && (e = hipSetDevice(device)) != hipSuccess) return e;
    void *ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (cur != device) (void)hipSetDevice(cur);
    if (e != hipSuccess) return e;
    if (!ptr) return hipErrorInvalidSymbol;
    g_scratch_ptr[device] = ptr;
    return hipSuccess;
}

void *noalloc_scratch(int device)
{
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return g_scratch_ptr[device];
}

}  // namespace irl
