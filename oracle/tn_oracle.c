/*
 * Plain CPU oracle for the temporal component matrix, the hashed proxies and
 * their recombination.  TEST INFRASTRUCTURE ONLY: the tests, the smoke check
 * and the CPU-baseline leg of the benchmark call it; the library's product
 * path never links, loads or calls it, and it shares no code with that path.
 *
 * Every routine is the definition written out, slow and unblocked:
 *   - component matrix, reverse time (Sec. 3.4 with the adjacency rule of
 *     Sec. 2.1): C <- I; for each distinct time step tau from the last to the
 *     first, every node x touched at tau gets
 *         new[x] = C[x] OR  OR_{(x,y) at tau} C[y]   (also (y,x) if undirected)
 *     computed from the rows as they were before tau, then all rows are
 *     replaced.  Events at the same time step are not adjacent (Sec. 2.1), so
 *     they never chain.  Row u of C is the out-component of u (the transpose
 *     of the paper's matrix S, whose columns are out-components, Sec. 3.1).
 *   - forward matrix S (Algorithm 1, Sec. 3.1): S <- I; for each time step in
 *     chronological order the same snapshot OR, information flowing from the
 *     source of an event to its target.
 *   - "sequential" mode: each event is its own time step in list order, the
 *     literal reading of Algorithm 1 on a time-ordered list.
 * Bit layout: node w is bit (w & 63) of word (w >> 6) of a row.  Every
 * routine can be restricted to a range of word columns [w0, w0 + nw): the
 * update only ORs rows, so each bit column evolves on its own.
 *
 * Hash family (Sec. 4.1): MultAddMod(x, acc, a) = (x * acc + a) mod (2^61-1)
 * with the exact 128-bit product; acc(i, x) starts at A(i,0) and is folded
 * with A(i,1..order-1); h(u) = (acc(0,x0) ^ acc(1,x1) ^ acc(2,x2)) mod K with
 * x0 / x1 the low / high 32 bits of u and x2 = x0 + x1.
 *
 * Recombination (Sec. 4.2, Eqs. DefInvHComp and DefEstOCMerge): the estimated
 * out-component of u is the set of nodes w with P_j[h_j(u)][h_j(w)] = 1 for
 * every hash j; the per-hash lifted size counts w with that bit set in hash j.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define TNO_MERSENNE61 ((((uint64_t)1) << 61) - 1)

static int popcount64(uint64_t x)
{
    int c = 0;
    while (x) {
        x &= x - 1;
        ++c;
    }
    return c;
}

static void set_identity(uint32_t n, int64_t w0, int64_t nw, uint64_t *M)
{
    memset(M, 0, sizeof(uint64_t) * (size_t)n * (size_t)nw);
    for (uint32_t u = 0; u < n; ++u) {
        int64_t word = (int64_t)(u >> 6);
        if (word >= w0 && word < w0 + nw)
            M[(size_t)u * nw + (size_t)(word - w0)] = ((uint64_t)1) << (u & 63);
    }
}

/*
 * One snapshot step over the events idx in [a, b): every touched node x gets
 * new[x] = M[x] | OR of M[y] over the events that carry information from y to
 * x, all computed from the old rows, then written back.
 * forward = 0: reverse-time rule, event (s, d) gives new[s] |= M[d].
 * forward = 1: chronological rule, event (s, d) gives new[d] |= M[s].
 * Undirected events carry information both ways.
 */
static int snapshot_step(int64_t a, int64_t b, const uint32_t *src,
                         const uint32_t *dst, int directed, int forward,
                         int64_t nw, uint64_t *M, int32_t *slot,
                         uint32_t *touched, uint64_t *newrows)
{
    int64_t k = 0;
    for (int64_t e = a; e < b; ++e) {
        uint32_t xs[2] = {src[e], dst[e]};
        for (int q = 0; q < 2; ++q) {
            uint32_t x = xs[q];
            if (slot[x] < 0) {
                slot[x] = (int32_t)k;
                touched[k] = x;
                memcpy(newrows + (size_t)k * nw, M + (size_t)x * nw,
                       sizeof(uint64_t) * (size_t)nw);
                ++k;
            }
        }
    }
    for (int64_t e = a; e < b; ++e) {
        uint32_t s = src[e], d = dst[e];
        uint32_t to = forward ? d : s;   /* row that receives */
        uint32_t from = forward ? s : d; /* row that is read  */
        uint64_t *r = newrows + (size_t)slot[to] * nw;
        const uint64_t *f = M + (size_t)from * nw;
        for (int64_t w = 0; w < nw; ++w)
            r[w] |= f[w];
        if (!directed) {
            uint64_t *r2 = newrows + (size_t)slot[from] * nw;
            const uint64_t *f2 = M + (size_t)to * nw;
            for (int64_t w = 0; w < nw; ++w)
                r2[w] |= f2[w];
        }
    }
    for (int64_t i = 0; i < k; ++i) {
        memcpy(M + (size_t)touched[i] * nw, newrows + (size_t)i * nw,
               sizeof(uint64_t) * (size_t)nw);
        slot[touched[i]] = -1;
    }
    return 0;
}

static int run_matrix(uint32_t n, int64_t m, const uint32_t *src,
                      const uint32_t *dst, const int64_t *t, int directed,
                      int sequential, int forward, int64_t w0, int64_t nw,
                      uint64_t *M)
{
    if (nw < 0 || w0 < 0)
        return -1;
    for (int64_t e = 0; e < m; ++e) {
        if (src[e] >= n || dst[e] >= n)
            return -2;
        if (e > 0 && t[e] < t[e - 1])
            return -3;
    }
    set_identity(n, w0, nw, M);
    if (m == 0 || nw == 0)
        return 0;
    /* largest group of equal time steps bounds the scratch */
    int64_t maxg = 1, run = 1;
    for (int64_t e = 1; e < m; ++e) {
        run = (t[e] == t[e - 1]) ? run + 1 : 1;
        if (run > maxg)
            maxg = run;
    }
    if (sequential)
        maxg = 1;
    int32_t *slot = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    uint32_t *touched = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(2 * maxg));
    uint64_t *newrows =
        (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(2 * maxg) * (size_t)nw);
    if (!slot || !touched || !newrows) {
        free(slot);
        free(touched);
        free(newrows);
        return -4;
    }
    for (uint32_t x = 0; x < n; ++x)
        slot[x] = -1;
    if (forward) {
        int64_t a = 0;
        while (a < m) {
            int64_t b = a + 1;
            if (!sequential)
                while (b < m && t[b] == t[a])
                    ++b;
            snapshot_step(a, b, src, dst, directed, 1, nw, M, slot, touched, newrows);
            a = b;
        }
    } else {
        int64_t b = m;
        while (b > 0) {
            int64_t a = b - 1;
            if (!sequential)
                while (a > 0 && t[a - 1] == t[b - 1])
                    --a;
            snapshot_step(a, b, src, dst, directed, 0, nw, M, slot, touched, newrows);
            b = a;
        }
    }
    free(slot);
    free(touched);
    free(newrows);
    return 0;
}

/* Reverse-time component matrix C restricted to word columns [w0, w0+nw);
 * C is n x nw words.  Returns 0, -2 for a node id >= n, -3 for decreasing t. */
int tno_reverse_matrix(uint32_t n, int64_t m, const uint32_t *src,
                       const uint32_t *dst, const int64_t *t, int directed,
                       int sequential, int64_t w0, int64_t nw, uint64_t *C)
{
    return run_matrix(n, m, src, dst, t, directed, sequential, 0, w0, nw, C);
}

/* Forward (chronological) matrix S of Algorithm 1 restricted to word columns
 * [w0, w0+nw).  Row x of S is the in-component of x, column u of S the
 * out-component of u. */
int tno_forward_matrix(uint32_t n, int64_t m, const uint32_t *src,
                       const uint32_t *dst, const int64_t *t, int directed,
                       int sequential, int64_t w0, int64_t nw, uint64_t *S)
{
    return run_matrix(n, m, src, dst, t, directed, sequential, 1, w0, nw, S);
}

/* Row popcounts: out[u] = number of ones in row u (n rows of nw words). */
void tno_row_counts(uint32_t n, int64_t nw, const uint64_t *M, int64_t *out)
{
    for (uint32_t u = 0; u < n; ++u) {
        int64_t c = 0;
        for (int64_t w = 0; w < nw; ++w)
            c += popcount64(M[(size_t)u * nw + (size_t)w]);
        out[u] = c;
    }
}

/* Column popcounts: col[b] = number of rows with bit b set, b < 64*nw. */
void tno_col_counts(uint32_t n, int64_t nw, const uint64_t *M, int64_t *col)
{
    for (int64_t b = 0; b < 64 * nw; ++b)
        col[b] = 0;
    for (uint32_t u = 0; u < n; ++u)
        for (int64_t b = 0; b < 64 * nw; ++b)
            col[b] += (int64_t)((M[(size_t)u * nw + (size_t)(b >> 6)] >> (b & 63)) & 1u);
}

/* (x * acc + a) mod (2^61 - 1) with the exact 128-bit product. */
uint64_t tno_multaddmod(uint64_t x, uint64_t acc, uint64_t a)
{
    unsigned __int128 r = (unsigned __int128)x * acc + a;
    return (uint64_t)(r % TNO_MERSENNE61);
}

/* acc(i, x) for one row A_i of the coefficient table (order entries). */
uint64_t tno_poly(const uint64_t *Ai, int order, uint64_t x)
{
    uint64_t acc = Ai[0] % TNO_MERSENNE61;
    for (int l = 1; l < order; ++l)
        acc = tno_multaddmod(x, acc, Ai[l]);
    return acc;
}

/* h(u) for one hash function with table A (3 rows of `order` entries). */
uint64_t tno_hash_raw(const uint64_t *A, int order, uint64_t u)
{
    uint64_t x0 = u & 0xffffffffu;
    uint64_t x1 = u >> 32;
    uint64_t x2 = x0 + x1;
    return tno_poly(A, order, x0) ^ tno_poly(A + order, order, x1) ^
           tno_poly(A + 2 * order, order, x2);
}

/* bucket[j*n + u] = h_j(u) mod K for H hash functions, A is H x 3 x order. */
void tno_hash_nodes(uint32_t n, uint32_t H, const uint64_t *A, int order,
                    uint32_t K, uint32_t *bucket)
{
    for (uint32_t j = 0; j < H; ++j)
        for (uint32_t u = 0; u < n; ++u)
            bucket[(size_t)j * n + u] =
                (uint32_t)(tno_hash_raw(A + (size_t)j * 3 * order, order, u) % K);
}

/*
 * Recombination for the sources us[0..ns): est[i] = #{w < n : for every j,
 * bit bucket_j(w) of row bucket_j(us[i]) of P_j is set}; lifted[j*ns + i] =
 * #{w < n : that bit is set in hash j}.  P is H matrices of K rows of ldK
 * words, bucket is H x n.
 */
void tno_recombine(uint32_t n, uint32_t H, uint32_t K, int64_t ldK,
                   const uint64_t *P, const uint32_t *bucket, int64_t ns,
                   const uint32_t *us, int64_t *est, int64_t *lifted)
{
    for (int64_t i = 0; i < ns; ++i) {
        uint32_t u = us[i];
        int64_t count = 0;
        for (uint32_t j = 0; j < H; ++j)
            lifted[(size_t)j * ns + i] = 0;
        for (uint32_t w = 0; w < n; ++w) {
            int all = 1;
            for (uint32_t j = 0; j < H; ++j) {
                const uint64_t *Pj = P + (size_t)j * K * ldK;
                uint32_t r = bucket[(size_t)j * n + u];
                uint32_t c = bucket[(size_t)j * n + w];
                int bit = (int)((Pj[(size_t)r * ldK + (c >> 6)] >> (c & 63)) & 1u);
                lifted[(size_t)j * ns + i] += bit;
                all &= bit;
            }
            count += all;
        }
        est[i] = count;
    }
}
