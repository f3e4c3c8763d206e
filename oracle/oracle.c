/*
 * CPU oracle for the SieveJoin hot path -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, single-threaded C. Nothing here is tuned; every routine follows the
 * definition it implements as literally as possible so that a reader can check it
 * against the paper (arXiv 2308.16370, "SieveJoin: Boosting Multi-Way Joins with
 * Reusable Bloom Filters") by eye. Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library; the GPU path never does.
 *
 * Contents
 *   1. Hash mixers (published definitions, see each function).
 *   2. The blocked Bloom filter: build (set bits) and probe (contains), i.e. the
 *      filter of Section 2.1 step 1 ("by the linear scanning and hashing of every
 *      tuple ... the corresponding bit ... is set to 1") in its cache-blocked form.
 *      The paper does not fix a hash family or bit pattern; the reading used here is:
 *        h     = fmix32((u32)key ^ seed)
 *        block = floor(h * nblocks / 2^32)
 *        g     = h * 0x9E3779B1 (mod 2^32),  g = g ^ (g >> 16)
 *        bit i = the top logB bits of g * M_i (mod 2^32), i = 0 .. k-1, k <= 12,
 *                with M_i the odd constants of bf_mult[] below
 *      i.e. k independent, uniformly placed bits inside one block of B bits (two
 *      of a key's bits may coincide). Block b occupies 32-bit words
 *      [b*B/32, (b+1)*B/32); bit p of a block is bit (p mod 32) of word (p / 32).
 *   3. The multi-way join result by a plain left-deep binary hash-join plan with no
 *      filters (the enumeration phase of Section 2.2 without pruning), sorted, plus
 *      its count and checksum.
 *
 * Parity pins for everything in this file live in tests/test_oracle_*.py.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ---------------------------------------------------------------- 1. mixers */

/* MurmurHash3 32-bit finaliser (Austin Appleby, public domain). */
uint32_t orc_fmix32(uint32_t h)
{
    h ^= h >> 16;
    h *= 0x85ebca6bu;
    h ^= h >> 13;
    h *= 0xc2b2ae35u;
    h ^= h >> 16;
    return h;
}

/* SplitMix64 output function (Steele, Lea and Flood, OOPSLA 2014). */
uint64_t orc_mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

/* Per-tuple checksum factor of relation i's row id: mix64((i << 32) | rid) | 1. */
uint64_t orc_chk_factor(uint32_t rel, uint32_t rid)
{
    return orc_mix64(((uint64_t)rel << 32) | (uint64_t)rid) | 1ull;
}

/* ------------------------------------------------------- 2. blocked Bloom filter */

/* Odd multipliers that spread the second hash word over the k bit positions. */
static const uint32_t bf_mult[12] = {
    0x85EBCA77u, 0xC2B2AE3Du, 0x27D4EB2Fu, 0x165667B1u, 0xD3A2646Du, 0xFD7046C5u,
    0xB55A4F09u, 0x2545F491u, 0x9E6C63D1u, 0x7FEB352Du, 0x846CA68Bu, 0x68E31DA5u,
};

/* The k bit positions (0..B-1) of `key` and the index of its block. */
static uint32_t bf_pattern(int32_t key, uint32_t nblocks, int k, int logB, uint32_t seed,
                           uint32_t *pos)
{
    uint32_t h = orc_fmix32((uint32_t)key ^ seed);
    uint32_t block = (uint32_t)(((uint64_t)h * (uint64_t)nblocks) >> 32);
    uint32_t g = h * 0x9E3779B1u;
    g ^= g >> 16;
    for (int i = 0; i < k; i++)
        pos[i] = (g * bf_mult[i]) >> (32 - logB);
    return block;
}

/* Number of blocks for n keys at bits_per_key: ceil(bpk * n / B), at least 1. */
uint64_t orc_bf_nblocks(uint64_t n, uint32_t bits_per_key, int logB)
{
    uint64_t B = 1ull << logB;
    uint64_t nb = (n * (uint64_t)bits_per_key + B - 1) / B;
    return nb ? nb : 1;
}

/* Block index and bit positions of one key (exported for the pattern tests). */
uint32_t orc_bf_pattern(int32_t key, uint32_t nblocks, int k, int logB, uint32_t seed,
                        uint32_t *pos_out)
{
    return bf_pattern(key, nblocks, k, logB, seed, pos_out);
}

/* Insert keys[rows[i]] (or keys[i] when rows is NULL) for i < n into the filter. */
void orc_bf_build(const int32_t *keys, const uint32_t *rows, int64_t n, uint32_t *words,
                  uint32_t nblocks, int k, int logB, uint32_t seed)
{
    uint32_t pos[64];
    uint32_t wpb = (1u << logB) / 32u;
    for (int64_t i = 0; i < n; i++) {
        int32_t key = rows ? keys[rows[i]] : keys[i];
        uint32_t b = bf_pattern(key, nblocks, k, logB, seed, pos);
        for (int j = 0; j < k; j++)
            words[(uint64_t)b * wpb + pos[j] / 32u] |= 1u << (pos[j] % 32u);
    }
}

/* out[i] = 1 when every bit of keys[rows[i]]'s pattern is set, else 0. */
void orc_bf_probe(const int32_t *keys, const uint32_t *rows, int64_t n, const uint32_t *words,
                  uint32_t nblocks, int k, int logB, uint32_t seed, uint8_t *out)
{
    uint32_t pos[64];
    uint32_t wpb = (1u << logB) / 32u;
    for (int64_t i = 0; i < n; i++) {
        int32_t key = rows ? keys[rows[i]] : keys[i];
        uint32_t b = bf_pattern(key, nblocks, k, logB, seed, pos);
        uint8_t hit = 1;
        for (int j = 0; j < k; j++)
            if (!(words[(uint64_t)b * wpb + pos[j] / 32u] & (1u << (pos[j] % 32u))))
                hit = 0;
        out[i] = hit;
    }
}

/* ------------------------------------------------- 3. binary hash-join plan */

/*
 * One join step s = 1..nsteps: bind relation child[s] through the equality
 *     R_child[child_col] == R_parent[parent_col]
 * where parent was bound by an earlier step (step 0 binds the root). After the
 * step, every closing equality listed for it is checked on the new tuples.
 *
 * Relations are given as flat arrays: nrows[r], the column pointer table
 * cols[r*maxcols + c], and the predicate (pred_col[r] < 0: none; keep
 * lo <= v < hi). Only the rows of `sel[r]` (ascending row ids, nsel[r] of them)
 * take part -- the caller evaluates the predicates.
 */
typedef struct {
    uint32_t *t;      /* tuples, row-major, width w */
    int64_t n, cap;
    int w;
} tupbuf;

static int tb_push(tupbuf *b, const uint32_t *src, int w, int slot, uint32_t rid)
{
    if (b->n == b->cap) {
        int64_t nc = b->cap ? b->cap * 2 : 1024;
        uint32_t *p = (uint32_t *)realloc(b->t, (size_t)nc * (size_t)w * sizeof(uint32_t));
        if (!p)
            return -1;
        b->t = p;
        b->cap = nc;
    }
    uint32_t *d = b->t + b->n * w;
    memcpy(d, src, (size_t)w * sizeof(uint32_t));
    d[slot] = rid;
    b->n++;
    return 0;
}

/* Chained hash table: distinct keys in open-addressed slots, rows chained in
 * ascending row-id order through next[]. */
typedef struct {
    int32_t *skey;
    int64_t *shead;   /* -1: empty slot */
    int64_t *next;    /* index into the selection, -1 ends a chain */
    uint64_t mask;
} chtab;

static uint64_t slot_of(int32_t key, uint64_t mask)
{
    return orc_mix64((uint64_t)(uint32_t)key) & mask;
}

static int ch_build(chtab *h, const int32_t *col, const uint32_t *sel, int64_t nsel)
{
    uint64_t cap = 16;
    while (cap < 2ull * (uint64_t)nsel + 1)
        cap <<= 1;
    h->mask = cap - 1;
    h->skey = (int32_t *)calloc(cap, sizeof(int32_t));
    h->shead = (int64_t *)malloc(cap * sizeof(int64_t));
    h->next = (int64_t *)malloc(((size_t)nsel + 1) * sizeof(int64_t));
    if (!h->skey || !h->shead || !h->next)
        return -1;
    for (uint64_t i = 0; i < cap; i++)
        h->shead[i] = -1;
    /* insert in descending order and push at the head: chains end up ascending */
    for (int64_t i = nsel - 1; i >= 0; i--) {
        int32_t key = col[sel[i]];
        uint64_t s = slot_of(key, h->mask);
        while (h->shead[s] >= 0 && h->skey[s] != key)
            s = (s + 1) & h->mask;
        if (h->shead[s] < 0)
            h->skey[s] = key;
        h->next[i] = h->shead[s];
        h->shead[s] = i;
    }
    return 0;
}

static int64_t ch_find(const chtab *h, int32_t key)
{
    uint64_t s = slot_of(key, h->mask);
    while (h->shead[s] >= 0) {
        if (h->skey[s] == key)
            return h->shead[s];
        s = (s + 1) & h->mask;
    }
    return -1;
}

static void ch_free(chtab *h)
{
    free(h->skey);
    free(h->shead);
    free(h->next);
}

static int cmp_w;
static int tuple_cmp(const void *a, const void *b)
{
    const uint32_t *x = (const uint32_t *)a, *y = (const uint32_t *)b;
    for (int i = 0; i < cmp_w; i++) {
        if (x[i] != y[i])
            return x[i] < y[i] ? -1 : 1;
    }
    return 0;
}

typedef struct {
    uint32_t *tuples;
    int64_t count;
    uint64_t checksum;
    int nrels;
} orc_result;

/*
 * Returns a heap result (free with orc_result_free) or NULL on allocation failure.
 *   nrels, maxcols, cols[nrels*maxcols], sel[nrels], nsel[nrels]
 *   root; nsteps = nrels-1; step arrays child/child_col/parent/parent_col [nsteps]
 *   nclose closing equalities (ca_rel, ca_col, cb_rel, cb_col), each applied after
 *   step close_after[i] (the first step where both relations are bound).
 */
orc_result *orc_hash_join(int nrels, int maxcols, const int32_t *const *cols,
                          const uint32_t *const *sel, const int64_t *nsel, int root,
                          const int *child, const int *child_col, const int *parent,
                          const int *parent_col, int nclose, const int *ca_rel,
                          const int *ca_col, const int *cb_rel, const int *cb_col,
                          const int *close_after)
{
    int w = nrels;
    tupbuf cur = {0}, nxt = {0};
    cur.w = nxt.w = w;
    uint32_t *zero = (uint32_t *)calloc((size_t)w, sizeof(uint32_t));
    orc_result *res = (orc_result *)calloc(1, sizeof(orc_result));
    if (!zero || !res)
        return NULL;
    for (int64_t i = 0; i < nsel[root]; i++)
        if (tb_push(&cur, zero, w, root, sel[root][i]))
            return NULL;
    for (int s = 0; s < nrels - 1; s++) {
        int c = child[s], cc = child_col[s], p = parent[s], pc = parent_col[s];
        const int32_t *ccol = cols[c * maxcols + cc];
        const int32_t *pcol = cols[p * maxcols + pc];
        chtab h;
        if (ch_build(&h, ccol, sel[c], nsel[c]))
            return NULL;
        nxt.n = 0;
        for (int64_t i = 0; i < cur.n; i++) {
            const uint32_t *t = cur.t + i * w;
            for (int64_t j = ch_find(&h, pcol[t[p]]); j >= 0; j = h.next[j]) {
                /* extend, then apply the closing equalities that become checkable */
                if (tb_push(&nxt, t, w, c, sel[c][j]))
                    return NULL;
                const uint32_t *u = nxt.t + (nxt.n - 1) * w;
                for (int e = 0; e < nclose; e++) {
                    if (close_after[e] != s)
                        continue;
                    int32_t va = cols[ca_rel[e] * maxcols + ca_col[e]][u[ca_rel[e]]];
                    int32_t vb = cols[cb_rel[e] * maxcols + cb_col[e]][u[cb_rel[e]]];
                    if (va != vb) {
                        nxt.n--;
                        break;
                    }
                }
            }
        }
        ch_free(&h);
        tupbuf tmp = cur;
        cur = nxt;
        nxt = tmp;
    }
    free(nxt.t);
    free(zero);
    cmp_w = w;
    if (cur.n > 1)
        qsort(cur.t, (size_t)cur.n, (size_t)w * sizeof(uint32_t), tuple_cmp);
    uint64_t chk = 0;
    for (int64_t i = 0; i < cur.n; i++) {
        uint64_t f = 1;
        for (int r = 0; r < w; r++)
            f *= orc_chk_factor((uint32_t)r, cur.t[i * w + r]);
        chk += f;
    }
    res->tuples = cur.t;
    res->count = cur.n;
    res->checksum = chk;
    res->nrels = w;
    return res;
}

int64_t orc_result_count(const orc_result *r) { return r->count; }
uint64_t orc_result_checksum(const orc_result *r) { return r->checksum; }
void orc_result_copy(const orc_result *r, uint32_t *out)
{
    if (r->count)
        memcpy(out, r->tuples, (size_t)r->count * (size_t)r->nrels * sizeof(uint32_t));
}
void orc_result_free(orc_result *r)
{
    if (r) {
        free(r->tuples);
        free(r);
    }
}

/* ---------------------------------------------------------------- 4. directed triangles */

/*
 * The cyclic query E1 join E2 join E3 on E1.dst = E2.src, E2.dst = E3.src,
 * E3.dst = E1.src over one edge list (the 3-cycle query of Section 2.3), counted by
 * adjacency intersection instead of a join plan: a result tuple is a choice of
 * edges e1 = (a -> b), e2 = (b -> c), e3 = (c -> a), so for every edge e1 the
 * tuples are the pairs (e2, e3) of an out-edge of b and an in-edge of a that meet in
 * the same vertex c. Both adjacency lists are sorted by that vertex and merged; a
 * vertex shared by several parallel edges contributes every pair. The checksum uses
 * relation indices 0, 1, 2 for E1, E2, E3 (the definition in Section 3 above).
 * E2 and E3 are the edge list (src, dst) of n rows; E1 is (e1_src, e1_dst) of m
 * rows: the same list, or a subset of rows (row ids then number the subset).
 */
typedef struct {
    int32_t key;   /* the vertex the list is grouped by */
    int32_t nbr;   /* the other end */
    uint32_t id;   /* edge row id */
} adj_t;

static int adj_cmp(const void *x, const void *y)
{
    const adj_t *a = (const adj_t *)x, *b = (const adj_t *)y;
    if (a->key != b->key) return a->key < b->key ? -1 : 1;
    if (a->nbr != b->nbr) return a->nbr < b->nbr ? -1 : 1;
    return a->id < b->id ? -1 : (a->id > b->id);
}

/* first index i in [lo, hi) with a[i].key >= key */
static int64_t adj_lower(const adj_t *a, int64_t lo, int64_t hi, int32_t key)
{
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (a[mid].key < key) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

/* first index i in [lo, hi) with a[i].key > key */
static int64_t adj_upper(const adj_t *a, int64_t lo, int64_t hi, int32_t key)
{
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (a[mid].key <= key) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

int orc_triangle_cycles(int64_t n, const int32_t *src, const int32_t *dst, int64_t m, const int32_t *e1_src,
                        const int32_t *e1_dst, int64_t *count, uint64_t *checksum)
{
    adj_t *out = (adj_t *)malloc((size_t)(n ? n : 1) * sizeof(adj_t));   /* grouped by src, nbr = dst */
    adj_t *in = (adj_t *)malloc((size_t)(n ? n : 1) * sizeof(adj_t));    /* grouped by dst, nbr = src */
    if (!out || !in) {
        free(out);
        free(in);
        return -1;
    }
    for (int64_t e = 0; e < n; ++e) {
        out[e].key = src[e]; out[e].nbr = dst[e]; out[e].id = (uint32_t)e;
        in[e].key = dst[e];  in[e].nbr = src[e];  in[e].id = (uint32_t)e;
    }
    qsort(out, (size_t)n, sizeof(adj_t), adj_cmp);
    qsort(in, (size_t)n, sizeof(adj_t), adj_cmp);
    int64_t cnt = 0;
    uint64_t chk = 0;
    for (int64_t e1 = 0; e1 < m; ++e1) {
        const int32_t a = e1_src[e1], b = e1_dst[e1];
        int64_t i = adj_lower(out, 0, n, b), ie = adj_upper(out, i, n, b);   /* out-edges of b */
        int64_t j = adj_lower(in, 0, n, a), je = adj_upper(in, j, n, a);     /* in-edges of a */
        const uint64_t f1 = orc_chk_factor(0, (uint32_t)e1);
        while (i < ie && j < je) {        /* out(b) by c = nbr, in(a) by c = nbr */
            const int32_t ci = out[i].nbr, cj = in[j].nbr;
            if (ci < cj) { ++i; continue; }
            if (cj < ci) { ++j; continue; }
            int64_t i2 = i, j2 = j;
            while (i2 < ie && out[i2].nbr == ci) ++i2;
            while (j2 < je && in[j2].nbr == ci) ++j2;
            for (int64_t x = i; x < i2; ++x)
                for (int64_t y = j; y < j2; ++y) {
                    ++cnt;
                    chk += f1 * orc_chk_factor(1, out[x].id) * orc_chk_factor(2, in[y].id);
                }
            i = i2;
            j = j2;
        }
    }
    free(out);
    free(in);
    *count = cnt;
    *checksum = chk;
    return 0;
}

/* ---------------------------------------------------------------- 5. 4-cliques */

/*
 * The 4-clique query over six binary relations (Section 3.1.3 runs it on an edge
 * list): relation XY holds pairs (x, y) of two of the four variables a, b, c, d, and
 * a result tuple is one row of each of AB, AC, AD, BC, BD, CD that agree on every
 * variable. Written as a generic join in the variable order a, b, c, d: for each AB
 * row (a, b), each AC row with that a gives c and each AD row with that a gives d;
 * BC, BD and CD then contribute every row holding (b, c), (b, d) and (c, d). Their
 * rows are grouped per pair (count and sum of checksum factors), so one lookup stands
 * for all of them. rel[6] are the relations' indices in the query (their checksum
 * factors); each relation comes as n rows of (x, y, row id), x the earlier variable.
 */
typedef struct {
    uint64_t key;   /* (x << 32) | y as unsigned words */
    uint64_t cnt;
    uint64_t fsum;
} pairagg_t;

static int u64_cmp(const void *x, const void *y)
{
    const uint64_t a = *(const uint64_t *)x, b = *(const uint64_t *)y;
    return a < b ? -1 : (a > b);
}

static uint64_t pair_of(int32_t x, int32_t y)
{
    return ((uint64_t)(uint32_t)x << 32) | (uint32_t)y;
}

/* rows grouped per pair; returns the number of distinct pairs, -1 on no memory */
static int64_t pairs_build(int64_t n, const int32_t *x, const int32_t *y, const uint32_t *id, uint32_t rel,
                           pairagg_t **out)
{
    uint64_t *tmp = (uint64_t *)malloc((size_t)(n ? n : 1) * 2 * sizeof(uint64_t));
    pairagg_t *p = (pairagg_t *)malloc((size_t)(n ? n : 1) * sizeof(pairagg_t));
    if (!tmp || !p) {
        free(tmp);
        free(p);
        return -1;
    }
    for (int64_t i = 0; i < n; ++i) {   /* (pair, factor) records sorted by pair */
        tmp[2 * i] = pair_of(x[i], y[i]);
        tmp[2 * i + 1] = orc_chk_factor(rel, id[i]);
    }
    qsort(tmp, (size_t)n, 2 * sizeof(uint64_t), u64_cmp);
    int64_t m = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (m == 0 || p[m - 1].key != tmp[2 * i]) {
            p[m].key = tmp[2 * i];
            p[m].cnt = 0;
            p[m].fsum = 0;
            ++m;
        }
        p[m - 1].cnt += 1;
        p[m - 1].fsum += tmp[2 * i + 1];
    }
    free(tmp);
    *out = p;
    return m;
}

static const pairagg_t *pairs_find(const pairagg_t *p, int64_t m, uint64_t key)
{
    int64_t lo = 0, hi = m;
    while (lo < hi) {
        const int64_t mid = lo + (hi - lo) / 2;
        if (p[mid].key < key) lo = mid + 1;
        else hi = mid;
    }
    return (lo < m && p[lo].key == key) ? &p[lo] : 0;
}

int orc_clique4(const int64_t *n, const int32_t *const *x, const int32_t *const *y, const uint32_t *const *id,
                const uint32_t *rel, int64_t *count, uint64_t *checksum)
{
    /* order: 0 AB, 1 AC, 2 AD, 3 BC, 4 BD, 5 CD */
    adj_t *ac = (adj_t *)malloc((size_t)(n[1] ? n[1] : 1) * sizeof(adj_t));
    adj_t *ad = (adj_t *)malloc((size_t)(n[2] ? n[2] : 1) * sizeof(adj_t));
    pairagg_t *bc = 0, *bd = 0, *cd = 0;
    const int64_t mbc = pairs_build(n[3], x[3], y[3], id[3], rel[3], &bc);
    const int64_t mbd = pairs_build(n[4], x[4], y[4], id[4], rel[4], &bd);
    const int64_t mcd = pairs_build(n[5], x[5], y[5], id[5], rel[5], &cd);
    int rc = -1;
    if (!ac || !ad || mbc < 0 || mbd < 0 || mcd < 0) goto done;
    for (int64_t i = 0; i < n[1]; ++i) {
        ac[i].key = x[1][i]; ac[i].nbr = y[1][i]; ac[i].id = id[1][i];
    }
    for (int64_t i = 0; i < n[2]; ++i) {
        ad[i].key = x[2][i]; ad[i].nbr = y[2][i]; ad[i].id = id[2][i];
    }
    qsort(ac, (size_t)n[1], sizeof(adj_t), adj_cmp);
    qsort(ad, (size_t)n[2], sizeof(adj_t), adj_cmp);
    int64_t cnt = 0;
    uint64_t chk = 0;
    for (int64_t r = 0; r < n[0]; ++r) {
        const int32_t a = x[0][r], b = y[0][r];
        const uint64_t f0 = orc_chk_factor(rel[0], id[0][r]);
        const int64_t i0 = adj_lower(ac, 0, n[1], a), i1 = adj_upper(ac, i0, n[1], a);
        const int64_t j0 = adj_lower(ad, 0, n[2], a), j1 = adj_upper(ad, j0, n[2], a);
        for (int64_t i = i0; i < i1; ++i) {
            const int32_t c = ac[i].nbr;
            const pairagg_t *pbc = pairs_find(bc, mbc, pair_of(b, c));
            if (!pbc) continue;
            const uint64_t f1 = f0 * orc_chk_factor(rel[1], ac[i].id) * pbc->fsum;
            for (int64_t j = j0; j < j1; ++j) {
                const int32_t d = ad[j].nbr;
                const pairagg_t *pbd = pairs_find(bd, mbd, pair_of(b, d));
                if (!pbd) continue;
                const pairagg_t *pcd = pairs_find(cd, mcd, pair_of(c, d));
                if (!pcd) continue;
                cnt += (int64_t)(pbc->cnt * pbd->cnt * pcd->cnt);
                chk += f1 * orc_chk_factor(rel[2], ad[j].id) * pbd->fsum * pcd->fsum;
            }
        }
    }
    *count = cnt;
    *checksum = chk;
    rc = 0;
done:
    free(ac);
    free(ad);
    free(bc);
    free(bd);
    free(cd);
    return rc;
}
