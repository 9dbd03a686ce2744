/*
 * Plain C Slater-Condon Hamiltonian apply u = H w on a sorted determinant set.
 *
 * TEST INFRASTRUCTURE ONLY (part of the CPU oracle).  Same rules and reading as
 * oracle/hamiltonian.py (Methods, "Wave Function Ansatz", Hamiltonian equation;
 * chemists' integrals (pq|rs), alpha spin-orbitals before beta, sign of
 * a+_a a_i = (-1)^(occupied between i and a)).  Written as a straightforward
 * row loop so it can run the full 853,776-determinant space on a CPU.  Lookup
 * of a target determinant is a binary search in the ascending key array.
 *
 *   keys : ascending uint64 keys (alpha orbital p at bit p, beta at bit 32+p)
 *   h    : n*n doubles, g : n^4 doubles, g[((p*n+q)*n+r)*n+s] = (pq|rs)
 *   rows : optional list of rows to compute (NULL: all rows)
 *
 * The apply is pinned against the Python oracle and the brute-force Fock-space
 * Hamiltonian in tests/test_oracle_hamiltonian.py; the row extraction
 * (oracle_sc_row, the CSR of capply.csr) element by element, pattern and sign,
 * against the brute force and the Python rows in tests/test_oracle_sc_row.py,
 * which also compiles copies of this file with planted mistakes.
 */
#include <stdint.h>
#include <stddef.h>

static int64_t find_key(const uint64_t *keys, int64_t ns, uint64_t k)
{
    int64_t lo = 0, hi = ns - 1;
    while (lo <= hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (keys[mid] == k) return mid;
        if (keys[mid] < k) lo = mid + 1; else hi = mid - 1;
    }
    return -1;
}

static int parity_between(uint32_t bits, int i, int a)
{
    int lo = i < a ? i : a, hi = i < a ? a : i;
    uint32_t mask = ((1u << hi) - 1u) & ~((1u << (lo + 1)) - 1u);
    return __builtin_popcount(bits & mask) & 1 ? -1 : 1;
}

#define G(p, q, r, s) g[(((size_t)(p) * n + (q)) * n + (r)) * n + (s)]

static double row_apply(int n, const double *h, const double *g, const uint64_t *keys,
                        int64_t ns, const double *w, uint64_t key)
{
    uint32_t al = (uint32_t)(key & 0xffffffffu), be = (uint32_t)(key >> 32);
    int oa[32], ob[32], va[32], vb[32], noa = 0, nob = 0, nva = 0, nvb = 0;
    for (int p = 0; p < n; ++p) {
        if (al >> p & 1u) oa[noa++] = p; else va[nva++] = p;
        if (be >> p & 1u) ob[nob++] = p; else vb[nvb++] = p;
    }
    int64_t self = find_key(keys, ns, key);
    double acc = 0.0;

    /* diagonal */
    double d = 0.0;
    for (int x = 0; x < noa; ++x) d += h[oa[x] * n + oa[x]];
    for (int x = 0; x < nob; ++x) d += h[ob[x] * n + ob[x]];
    for (int x = 0; x < noa; ++x)
        for (int y = 0; y < noa; ++y)
            d += 0.5 * (G(oa[x], oa[x], oa[y], oa[y]) - G(oa[x], oa[y], oa[y], oa[x]));
    for (int x = 0; x < nob; ++x)
        for (int y = 0; y < nob; ++y)
            d += 0.5 * (G(ob[x], ob[x], ob[y], ob[y]) - G(ob[x], ob[y], ob[y], ob[x]));
    for (int x = 0; x < noa; ++x)
        for (int y = 0; y < nob; ++y)
            d += G(oa[x], oa[x], ob[y], ob[y]);
    acc += d * w[self];

    for (int spin = 0; spin < 2; ++spin) {
        const int *os = spin ? ob : oa, *oo = spin ? oa : ob, *vs = spin ? vb : va;
        int nos = spin ? nob : noa, noo = spin ? noa : nob, nvs = spin ? nvb : nva;
        uint32_t bits = spin ? be : al;
        /* singles */
        for (int x = 0; x < nos; ++x)
            for (int u = 0; u < nvs; ++u) {
                int i = os[x], a = vs[u];
                double v = h[i * n + a];
                for (int y = 0; y < nos; ++y) v += G(i, a, os[y], os[y]) - G(i, os[y], os[y], a);
                for (int y = 0; y < noo; ++y) v += G(i, a, oo[y], oo[y]);
                uint32_t nb = (bits & ~(1u << i)) | (1u << a);
                uint64_t t = spin ? ((uint64_t)al | ((uint64_t)nb << 32))
                                  : ((uint64_t)nb | ((uint64_t)be << 32));
                int64_t r = find_key(keys, ns, t);
                if (r >= 0) acc += parity_between(bits, i, a) * v * w[r];
            }
        /* same-spin doubles, i<j -> a<b, i->a then j->b */
        for (int x = 0; x < nos; ++x)
            for (int y = x + 1; y < nos; ++y)
                for (int u = 0; u < nvs; ++u)
                    for (int z = u + 1; z < nvs; ++z) {
                        int i = os[x], j = os[y], a = vs[u], b = vs[z];
                        int s1 = parity_between(bits, i, a);
                        uint32_t b1 = (bits & ~(1u << i)) | (1u << a);
                        int s2 = parity_between(b1, j, b);
                        uint32_t b2 = (b1 & ~(1u << j)) | (1u << b);
                        uint64_t t = spin ? ((uint64_t)al | ((uint64_t)b2 << 32))
                                          : ((uint64_t)b2 | ((uint64_t)be << 32));
                        int64_t r = find_key(keys, ns, t);
                        if (r >= 0)
                            acc += s1 * s2 * (G(i, a, j, b) - G(i, b, j, a)) * w[r];
                    }
    }
    /* opposite-spin doubles */
    for (int x = 0; x < noa; ++x)
        for (int u = 0; u < nva; ++u) {
            int i = oa[x], a = va[u];
            int s1 = parity_between(al, i, a);
            uint32_t a1 = (al & ~(1u << i)) | (1u << a);
            for (int y = 0; y < nob; ++y)
                for (int z = 0; z < nvb; ++z) {
                    int j = ob[y], b = vb[z];
                    int s2 = parity_between(be, j, b);
                    uint32_t b1 = (be & ~(1u << j)) | (1u << b);
                    int64_t r = find_key(keys, ns, (uint64_t)a1 | ((uint64_t)b1 << 32));
                    if (r >= 0) acc += s1 * s2 * G(i, a, j, b) * w[r];
                }
        }
    return acc;
}

/* u[k] = (H w)[rows[k]] for k < nrows, or u = H w when rows == NULL. */
void oracle_sc_apply(int n, const double *h, const double *g, const uint64_t *keys,
                     int64_t ns, const double *w, double *u, const int64_t *rows,
                     int64_t nrows)
{
    int64_t cnt = rows ? nrows : ns;
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t k = 0; k < cnt; ++k) {
        int64_t r = rows ? rows[k] : k;
        u[k] = row_apply(n, h, g, keys, ns, w, keys[r]);
    }
}

/* Connections of one row inside the set (diagonal first, then every single
 * and double that lands in the set, in enumeration order; duplicates cannot
 * occur).  Writes up to cap (col, value) pairs, returns the count. */
int64_t oracle_sc_row(int n, const double *h, const double *g, const uint64_t *keys, int64_t ns,
                      int64_t row, int64_t *cols, double *vals, int64_t cap)
{
    uint64_t key = keys[row];
    uint32_t al = (uint32_t)(key & 0xffffffffu), be = (uint32_t)(key >> 32);
    int oa[32], ob[32], va[32], vb[32], noa = 0, nob = 0, nva = 0, nvb = 0;
    for (int p = 0; p < n; ++p) {
        if (al >> p & 1u) oa[noa++] = p; else va[nva++] = p;
        if (be >> p & 1u) ob[nob++] = p; else vb[nvb++] = p;
    }
    int64_t c = 0;
#define EMIT(col, val) do { if (c < cap) { cols[c] = (col); vals[c] = (val); } ++c; } while (0)
    double d = 0.0;
    for (int x = 0; x < noa; ++x) d += h[oa[x] * n + oa[x]];
    for (int x = 0; x < nob; ++x) d += h[ob[x] * n + ob[x]];
    for (int x = 0; x < noa; ++x)
        for (int y = 0; y < noa; ++y)
            d += 0.5 * (G(oa[x], oa[x], oa[y], oa[y]) - G(oa[x], oa[y], oa[y], oa[x]));
    for (int x = 0; x < nob; ++x)
        for (int y = 0; y < nob; ++y)
            d += 0.5 * (G(ob[x], ob[x], ob[y], ob[y]) - G(ob[x], ob[y], ob[y], ob[x]));
    for (int x = 0; x < noa; ++x)
        for (int y = 0; y < nob; ++y)
            d += G(oa[x], oa[x], ob[y], ob[y]);
    EMIT(row, d);
    for (int spin = 0; spin < 2; ++spin) {
        const int *os = spin ? ob : oa, *oo = spin ? oa : ob, *vs = spin ? vb : va;
        int nos = spin ? nob : noa, noo = spin ? noa : nob, nvs = spin ? nvb : nva;
        uint32_t bits = spin ? be : al;
        for (int x = 0; x < nos; ++x)
            for (int u = 0; u < nvs; ++u) {
                int i = os[x], a = vs[u];
                uint32_t nb = (bits & ~(1u << i)) | (1u << a);
                uint64_t t = spin ? ((uint64_t)al | ((uint64_t)nb << 32))
                                  : ((uint64_t)nb | ((uint64_t)be << 32));
                int64_t r = find_key(keys, ns, t);
                if (r < 0) continue;
                double v = h[i * n + a];
                for (int y = 0; y < nos; ++y) v += G(i, a, os[y], os[y]) - G(i, os[y], os[y], a);
                for (int y = 0; y < noo; ++y) v += G(i, a, oo[y], oo[y]);
                EMIT(r, parity_between(bits, i, a) * v);
            }
        for (int x = 0; x < nos; ++x)
            for (int y = x + 1; y < nos; ++y)
                for (int u = 0; u < nvs; ++u)
                    for (int z = u + 1; z < nvs; ++z) {
                        int i = os[x], j = os[y], a = vs[u], b = vs[z];
                        int s1 = parity_between(bits, i, a);
                        uint32_t b1 = (bits & ~(1u << i)) | (1u << a);
                        int s2 = parity_between(b1, j, b);
                        uint32_t b2 = (b1 & ~(1u << j)) | (1u << b);
                        uint64_t t = spin ? ((uint64_t)al | ((uint64_t)b2 << 32))
                                          : ((uint64_t)b2 | ((uint64_t)be << 32));
                        int64_t r = find_key(keys, ns, t);
                        if (r >= 0) EMIT(r, s1 * s2 * (G(i, a, j, b) - G(i, b, j, a)));
                    }
    }
    for (int x = 0; x < noa; ++x)
        for (int u = 0; u < nva; ++u) {
            int i = oa[x], a = va[u];
            int s1 = parity_between(al, i, a);
            uint32_t a1 = (al & ~(1u << i)) | (1u << a);
            for (int y = 0; y < nob; ++y)
                for (int z = 0; z < nvb; ++z) {
                    int j = ob[y], b = vb[z];
                    int s2 = parity_between(be, j, b);
                    uint32_t b1 = (be & ~(1u << j)) | (1u << b);
                    int64_t r = find_key(keys, ns, (uint64_t)a1 | ((uint64_t)b1 << 32));
                    if (r >= 0) EMIT(r, s1 * s2 * G(i, a, j, b));
                }
        }
#undef EMIT
    (void)0;
    return c;
}
