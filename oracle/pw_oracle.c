/*
 * CPU oracle for the ProbeWalk estimator -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg may
 * load this file's library. It shares no code with the HIP path; the two meet
 * only in the seeded inputs and in the conventions written out below.
 *
 * What it computes (paper section 3, Algorithm 1 "ProbeWalk"):
 *   for each probe k = 0..K-1                                  (Alg. 1 outer loop)
 *     for each replica p = 0..R-1                              (Alg. 1 replica loop)
 *       a = sum_{i=0..L} z_{X_i}/d_{X_i}   over a walk X from s  (eq. for phi-hat)
 *       b = same over an independent walk from t
 *       U_p = a - b
 *     S1 = sum_p U_p,  S2 = sum_p U_p^2,  Q_k = (S1^2 - S2)/(R(R-1))  (U-statistic)
 *   G blocks of B consecutive probes; block means; median    (median-of-means)
 *
 * Walk sharing (an extension the paper does not make; off when M = 1): the
 * probes of each block are taken in groups of M consecutive probes (the last
 * group of a block may be smaller); all probes of a group are scored on the
 * same R walk pairs, whose random streams are keyed by the group's first
 * probe index. Groups never cross a block, so the G block means stay
 * independent, and each Q_k is still unbiased (its walks are independent of
 * its probe). With M = 1 this is Algorithm 1 exactly.
 *
 * Conventions this oracle fixes where the paper leaves freedom (each is a
 * reading of the paper, the GPU path implements the same reading on its own):
 *   - Randomness: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11), key =
 *     64-bit seed (low word first). Walk step i >= 1 uses word (i-1)&3 of the
 *     block with counter ((i-1)>>2, p, k, (uid<<1)|side); side 0 = s, 1 = t.
 *     Probe k's key material uses counters (j, 0xFFFFFFFF, k, uid<<1), j=0,1,2:
 *     block 0 -> round keys K0..K3; block 1 -> K4, K5, a_k = 1 + w2 mod (p-1),
 *     b_k = w3 mod p; block 2 -> coin = w0 & 1.
 *   - Neighbour choice (uniform over N(x), Alg. 1): j = floor(u*d_x / 2^32)
 *     into the ascending neighbour list.
 *   - Probe (Definition of the Paired-Sign Probe and its stateless
 *     generator, section 3.3): pi_k is a 6-round alternating Feistel network
 *     on Z_A x Z_{2^rb} (rb = floor(ceil(log2 n)/2), A = ceil(n/2^rb)) with
 *     cycle walking into [n]; r = 1 for odd n, else 2*coin; z_i = 0 when
 *     pi_k(i) >= n-r, else (-1)^(h_k(pi_k(i)>>1) + pi_k(i)) with
 *     h_k(u) = ((a_k u + b_k) mod p) mod 2, p = 2^31-1.
 *   - Per-walk sums in binary32: inv(x) = 1.0f/(float)d_x, a term is added
 *     only when z != 0, starting from +0.0f, in step order.
 *   - Per-probe sums are exact: every U_p is an integer multiple of 2^-54, so
 *     S1 is held as the integer S1*2^54; S2 is held as sum_p floor(U_p^2 2^64).
 *     Q_k is then formed in binary64 and stored as trunc(Q_k 2^64); block
 *     sums are exact integers, block means binary64. Summation order
 *     therefore never changes a result.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef __int128 i128;
typedef unsigned __int128 u128;

#define HASH_P 2147483647u /* 2^31 - 1 */

/* ------------------------------------------------------------------------ */
/* Philox4x32-10                                                             */
/* ------------------------------------------------------------------------ */
static void philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; round++) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

void pwo_philox(const uint32_t* ctr, const uint32_t* key, uint32_t* out)
{
    philox4x32_10(ctr, key, out);
}

/* ------------------------------------------------------------------------ */
/* Paired-Sign Probe, stateless generator                                   */
/* ------------------------------------------------------------------------ */
typedef struct {
    uint32_t n;      /* number of nodes */
    uint32_t rb;     /* bits of the XOR half */
    uint32_t A;      /* modulus of the additive half */
} domain_t;

#define FEISTEL_ROUNDS 6

typedef struct {
    uint32_t K[FEISTEL_ROUNDS]; /* Feistel round keys */
    uint32_t a, b;   /* hash parameters, a in [1,p-1], b in [0,p-1] */
    uint32_t r;      /* number of zero entries */
} probe_t;

static domain_t make_domain(uint32_t n)
{
    domain_t d;
    uint32_t w = 0;
    while (((uint64_t)1 << w) < n) w++;
    d.n = n;
    d.rb = w >> 1;
    d.A = (uint32_t)((n + ((1u << d.rb) - 1)) >> d.rb);
    return d;
}

static void make_probe(uint64_t seed, uint32_t uid, uint32_t k, uint32_t n, probe_t* pr)
{
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t c[4] = {0u, 0xFFFFFFFFu, k, uid << 1};
    uint32_t w[4];
    philox4x32_10(c, key, w);
    pr->K[0] = w[0]; pr->K[1] = w[1]; pr->K[2] = w[2]; pr->K[3] = w[3];
    c[0] = 1u;
    philox4x32_10(c, key, w);
    pr->K[4] = w[0]; pr->K[5] = w[1];
    pr->a = 1u + w[2] % (HASH_P - 1u);
    pr->b = w[3] % HASH_P;
    c[0] = 2u;
    philox4x32_10(c, key, w);
    uint32_t coin = w[0] & 1u;
    pr->r = (n & 1u) ? 1u : 2u * coin;
}

/* low 32 bits of the product of the low 24 bits of each operand */
static uint32_t mul24(uint32_t a, uint32_t b)
{
    return (uint32_t)((uint64_t)(a & 0xFFFFFFu) * (uint64_t)(b & 0xFFFFFFu));
}

/* bits 32..47 of the product of the low 24 bits of each operand */
static uint32_t mulhi24(uint32_t a, uint32_t b)
{
    return (uint32_t)(((uint64_t)(a & 0xFFFFFFu) * (uint64_t)(b & 0xFFFFFFu)) >> 32);
}

/* Feistel round function: two 24-bit multiplicative mixes with an xorshift */
static uint32_t fmix(uint32_t v, uint32_t key)
{
    uint32_t h = mul24(v ^ key, 0x9E3779u);
    h ^= h >> 15;
    return mul24(h, 0x873593u);
}

/* the permutation pi_k of [n] */
static uint32_t feistel_pi(const domain_t* d, const probe_t* pr, uint32_t x)
{
    const uint32_t mask = (1u << d->rb) - 1u;
    do {
        uint32_t L = x >> d->rb;
        uint32_t R = x & mask;
        for (int round = 0; round < FEISTEL_ROUNDS; round++) {
            uint32_t h;
            if ((round & 1) == 0) {
                /* additive half: L <- (L + F(R)) mod A with F(R) in [0, A) */
                h = fmix(R, pr->K[round]);
                uint32_t f = mulhi24(h >> 8, d->A << 8);
                L = L + f;
                if (L >= d->A) L -= d->A;
            } else if (d->rb > 0) {
                /* XOR half: R <- R xor (top rb bits of F(L)) */
                h = fmix(L, pr->K[round]);
                R ^= h >> (32u - d->rb);
            }
        }
        x = (L << d->rb) | R;
    } while (x >= d->n);
    return x;
}

static uint32_t hash_bit(const probe_t* pr, uint32_t u)
{
    uint64_t v = (uint64_t)pr->a * (uint64_t)u + (uint64_t)pr->b;
    return (uint32_t)(v % HASH_P) & 1u;
}

/* z^(k)_x in {-1, 0, +1} */
static int probe_z(const domain_t* d, const probe_t* pr, uint32_t x)
{
    uint32_t y = feistel_pi(d, pr, x);
    if (y >= d->n - pr->r) return 0;
    uint32_t bit = hash_bit(pr, y >> 1) ^ (y & 1u);
    return bit ? -1 : 1;
}

/* Evaluate pi_k (and z) for a list of nodes: used by the probe tests. */
void pwo_probe_eval(uint32_t n, uint64_t seed, uint32_t uid, uint32_t k,
                    int64_t count, const uint32_t* nodes, uint32_t* pi_out, int8_t* z_out,
                    uint32_t* params_out /* 9 words: K0..K5, a, b, r; may be NULL */)
{
    domain_t d = make_domain(n);
    probe_t pr;
    make_probe(seed, uid, k, n, &pr);
    for (int64_t i = 0; i < count; i++) {
        uint32_t y = feistel_pi(&d, &pr, nodes[i]);
        if (pi_out) pi_out[i] = y;
        if (z_out) z_out[i] = (int8_t)probe_z(&d, &pr, nodes[i]);
    }
    if (params_out) {
        for (int i = 0; i < FEISTEL_ROUNDS; i++) params_out[i] = pr.K[i];
        params_out[6] = pr.a; params_out[7] = pr.b; params_out[8] = pr.r;
    }
}

/* ------------------------------------------------------------------------ */
/* Walks                                                                     */
/* ------------------------------------------------------------------------ */
typedef struct {
    uint32_t n;
    const int64_t* row_ptr;
    const int32_t* col;
    float* inv;         /* 1.0f/(float)d_x */
} graph_t;

static float walk_sum(const graph_t* g, const domain_t* d, const probe_t* pr,
                      uint32_t start, int32_t L, uint64_t seed, uint32_t uid,
                      uint32_t k, uint32_t p, uint32_t side, int32_t* trace)
{
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t x = start;
    float acc = 0.0f;
    int z = probe_z(d, pr, x);
    if (z > 0) acc = acc + g->inv[x];
    else if (z < 0) acc = acc - g->inv[x];
    if (trace) trace[0] = (int32_t)x;
    uint32_t words[4] = {0, 0, 0, 0};
    for (int32_t i = 1; i <= L; i++) {
        uint32_t step = (uint32_t)(i - 1);
        if ((step & 3u) == 0u) {
            uint32_t c[4] = {step >> 2, p, k, (uid << 1) | side};
            philox4x32_10(c, key, words);
        }
        uint32_t u = words[step & 3u];
        uint64_t deg = (uint64_t)(g->row_ptr[x + 1] - g->row_ptr[x]);
        uint64_t j = ((uint64_t)u * deg) >> 32;
        x = (uint32_t)g->col[g->row_ptr[x] + (int64_t)j];
        z = probe_z(d, pr, x);
        if (z > 0) acc = acc + g->inv[x];
        else if (z < 0) acc = acc - g->inv[x];
        if (trace) trace[i] = (int32_t)x;
    }
    return acc;
}

/* The sums of m probes over one walk: acc[j] = sum_i z^(j)_{X_i}/d_{X_i}, each in
 * binary32 in step order, the walk's stream keyed by kwalk. */
static void walk_sums(const graph_t* g, const domain_t* d, const probe_t* prs, int m,
                      uint32_t start, int32_t L, uint64_t seed, uint32_t uid,
                      uint32_t kwalk, uint32_t p, uint32_t side, float* acc)
{
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t x = start;
    for (int j = 0; j < m; j++) {
        acc[j] = 0.0f;
        int z = probe_z(d, &prs[j], x);
        if (z > 0) acc[j] = acc[j] + g->inv[x];
        else if (z < 0) acc[j] = acc[j] - g->inv[x];
    }
    uint32_t words[4] = {0, 0, 0, 0};
    for (int32_t i = 1; i <= L; i++) {
        uint32_t step = (uint32_t)(i - 1);
        if ((step & 3u) == 0u) {
            uint32_t c[4] = {step >> 2, p, kwalk, (uid << 1) | side};
            philox4x32_10(c, key, words);
        }
        uint32_t u = words[step & 3u];
        uint64_t deg = (uint64_t)(g->row_ptr[x + 1] - g->row_ptr[x]);
        uint64_t jn = ((uint64_t)u * deg) >> 32;
        x = (uint32_t)g->col[g->row_ptr[x] + (int64_t)jn];
        for (int j = 0; j < m; j++) {
            int z = probe_z(d, &prs[j], x);
            if (z > 0) acc[j] = acc[j] + g->inv[x];
            else if (z < 0) acc[j] = acc[j] - g->inv[x];
        }
    }
}

/* First probe of the walk-sharing group that holds probe k (blocks of B, groups of M). */
static int64_t group_first(int64_t k, int64_t B, int64_t M)
{
    int64_t blk = k / B;
    return blk * B + ((k - blk * B) / M) * M;
}

void pwo_walk_trace(uint32_t n, const int64_t* row_ptr, const int32_t* col,
                    uint32_t start, int32_t L, uint64_t seed, uint32_t uid,
                    uint32_t k, uint32_t p, uint32_t side, int32_t* trace, float* acc_out)
{
    graph_t g = {n, row_ptr, col, NULL};
    g.inv = (float*)malloc(sizeof(float) * n);
    for (uint32_t v = 0; v < n; v++) g.inv[v] = 1.0f / (float)(row_ptr[v + 1] - row_ptr[v]);
    domain_t d = make_domain(n);
    probe_t pr;
    make_probe(seed, uid, k, n, &pr);
    float a = walk_sum(&g, &d, &pr, start, L, seed, uid, k, p, side, trace);
    if (acc_out) *acc_out = a;
    free(g.inv);
}

/* ------------------------------------------------------------------------ */
/* Fixed-point sums                                                          */
/* ------------------------------------------------------------------------ */

/* U * 2^54 as an integer; U is always an integer multiple of 2^-54 */
static i128 fix54(float U)
{
    double v = ldexp((double)U, 54);
    if (floor(v) != v) {
        fprintf(stderr, "pw_oracle: U=%a is not a multiple of 2^-54\n", (double)U);
        abort();
    }
    return (i128)v;
}

/* floor(U^2 * 2^64) */
static u128 sqfix64(float U)
{
    double sq = (double)U * (double)U; /* exact: 48 significant bits */
    return (u128)floor(ldexp(sq, 64));
}

/* per-probe statistic from the exact sums */
static double probe_q(i128 S1, u128 S2, int64_t R)
{
    double s1 = ldexp((double)S1, -54);
    double s2 = ldexp((double)S2, -64);
    double num = s1 * s1 - s2;
    double den = (double)R * (double)(R - 1);
    return num / den;
}

static int cmp_double(const void* a, const void* b)
{
    double x = *(const double*)a, y = *(const double*)b;
    return (x > y) - (x < y);
}

/* ------------------------------------------------------------------------ */
/* One query, Algorithm 1                                                    */
/* ------------------------------------------------------------------------ */
typedef struct {
    int32_t s, t, L;
    uint32_t uid;
    int64_t K, R, B, G;
    int64_t M;              /* walk-sharing group size (1 = none) */
    int64_t k_begin, k_end; /* probe range to run (sampling); [0, K) for a full query */
    double beta;
    double* q_out;      /* optional, K entries */
    double* ybar_out;   /* optional, G entries */
} query_t;

static void run_query(const graph_t* g, uint64_t seed, query_t* q)
{
    domain_t d = make_domain(g->n);
    i128* block_sum = (i128*)calloc((size_t)q->G, sizeof(i128));
    const int64_t M = q->M;
    probe_t* prs = (probe_t*)malloc(sizeof(probe_t) * (size_t)M);
    i128* S1 = (i128*)malloc(sizeof(i128) * (size_t)M);
    u128* S2 = (u128*)malloc(sizeof(u128) * (size_t)M);
    float* a = (float*)malloc(sizeof(float) * (size_t)M);
    float* b = (float*)malloc(sizeof(float) * (size_t)M);
    /* groups of M consecutive probes inside each block; k_end cuts at a group */
    for (int64_t k0 = q->k_begin; k0 < q->k_end;) {
        const int64_t blk_end = (k0 / q->B + 1) * q->B;
        const int m = (int)(M < blk_end - k0 ? M : blk_end - k0);
        for (int j = 0; j < m; j++) {
            make_probe(seed, q->uid, (uint32_t)(k0 + j), g->n, &prs[j]);
            S1[j] = 0;
            S2[j] = 0;
        }
        for (int64_t p = 0; p < q->R; p++) {
            walk_sums(g, &d, prs, m, (uint32_t)q->s, q->L, seed, q->uid, (uint32_t)k0, (uint32_t)p, 0u, a);
            walk_sums(g, &d, prs, m, (uint32_t)q->t, q->L, seed, q->uid, (uint32_t)k0, (uint32_t)p, 1u, b);
            for (int j = 0; j < m; j++) {
                float U = a[j] - b[j];
                S1[j] += fix54(U);
                S2[j] += sqfix64(U);
            }
        }
        for (int j = 0; j < m; j++) {
            double Q = probe_q(S1[j], S2[j], q->R);
            if (q->q_out) q->q_out[k0 + j] = Q;
            i128 Qfix = (i128)ldexp(Q, 64); /* truncation toward zero */
            block_sum[(k0 + j) / q->B] += Qfix;
        }
        k0 += m;
    }
    free(prs);
    free(S1);
    free(S2);
    free(a);
    free(b);
    double* ybar = (double*)malloc(sizeof(double) * (size_t)q->G);
    for (int64_t gi = 0; gi < q->G; gi++)
        ybar[gi] = ldexp((double)block_sum[gi], -64) / (double)q->B;
    if (q->ybar_out) memcpy(q->ybar_out, ybar, sizeof(double) * (size_t)q->G);
    qsort(ybar, (size_t)q->G, sizeof(double), cmp_double);
    if (q->G & 1) q->beta = ybar[q->G / 2];
    else q->beta = 0.5 * (ybar[q->G / 2 - 1] + ybar[q->G / 2]);
    free(ybar);
    free(block_sum);
}

typedef struct {
    const graph_t* g;
    uint64_t seed;
    query_t* qs;
    int64_t nq;
    int64_t next;
    pthread_mutex_t mu;
} pool_t;

static void* worker(void* arg)
{
    pool_t* pool = (pool_t*)arg;
    for (;;) {
        pthread_mutex_lock(&pool->mu);
        int64_t i = pool->next++;
        pthread_mutex_unlock(&pool->mu);
        if (i >= pool->nq) break;
        run_query(pool->g, pool->seed, &pool->qs[i]);
    }
    return NULL;
}

/*
 * Estimate a batch of queries; one query per thread at a time.
 *   K, R, B, G: per-query walk counts (the planner lives on the Python side).
 *   M:  per-query walk-sharing group size (NULL = 1 for all: Algorithm 1).
 *   k_end: per-query number of probes actually run (k_end == K for a full
 *          query; smaller values time a sample of the probes; whole groups).
 *   q_out: optional K-entry array per query for query 0 only (may be NULL).
 */
int pwo_estimate(uint32_t n, const int64_t* row_ptr, const int32_t* col,
                 int64_t nq, const int32_t* s, const int32_t* t, const int32_t* L,
                 const uint32_t* uid, const int64_t* K, const int64_t* R,
                 const int64_t* B, const int64_t* G, const int64_t* M, const int64_t* k_end,
                 uint64_t seed, int nthreads, double* beta_out,
                 double* q_out0, double* ybar_out0)
{
    graph_t g = {n, row_ptr, col, NULL};
    g.inv = (float*)malloc(sizeof(float) * n);
    for (uint32_t v = 0; v < n; v++) g.inv[v] = 1.0f / (float)(row_ptr[v + 1] - row_ptr[v]);
    query_t* qs = (query_t*)calloc((size_t)nq, sizeof(query_t));
    for (int64_t i = 0; i < nq; i++) {
        qs[i].s = s[i]; qs[i].t = t[i]; qs[i].L = L[i];
        qs[i].uid = uid ? uid[i] : (uint32_t)i;
        qs[i].K = K[i]; qs[i].R = R[i]; qs[i].B = B[i]; qs[i].G = G[i];
        qs[i].M = (M && M[i] > 1) ? M[i] : 1;
        qs[i].k_begin = 0;
        qs[i].k_end = k_end ? k_end[i] : K[i];
        qs[i].q_out = (i == 0) ? q_out0 : NULL;
        qs[i].ybar_out = (i == 0) ? ybar_out0 : NULL;
    }
    pool_t pool = {&g, seed, qs, nq, 0, PTHREAD_MUTEX_INITIALIZER};
    if (nthreads < 1) nthreads = 1;
    if (nthreads > nq) nthreads = (int)nq;
    pthread_t* th = (pthread_t*)malloc(sizeof(pthread_t) * (size_t)nthreads);
    for (int i = 0; i < nthreads; i++) pthread_create(&th[i], NULL, worker, &pool);
    for (int i = 0; i < nthreads; i++) pthread_join(th[i], NULL);
    for (int64_t i = 0; i < nq; i++) beta_out[i] = qs[i].beta;
    free(th);
    free(qs);
    free(g.inv);
    return 0;
}

/* The per-replica difference U_p for one (k, p): used by statistical tests. */
void pwo_replicas(uint32_t n, const int64_t* row_ptr, const int32_t* col,
                  int32_t s, int32_t t, int32_t L, uint32_t uid, uint32_t k,
                  int64_t p_begin, int64_t count, uint64_t seed, float* U_out)
{
    graph_t g = {n, row_ptr, col, NULL};
    g.inv = (float*)malloc(sizeof(float) * n);
    for (uint32_t v = 0; v < n; v++) g.inv[v] = 1.0f / (float)(row_ptr[v + 1] - row_ptr[v]);
    domain_t d = make_domain(n);
    probe_t pr;
    make_probe(seed, uid, k, n, &pr);
    for (int64_t i = 0; i < count; i++) {
        uint32_t p = (uint32_t)(p_begin + i);
        float a = walk_sum(&g, &d, &pr, (uint32_t)s, L, seed, uid, k, p, 0u, NULL);
        float b = walk_sum(&g, &d, &pr, (uint32_t)t, L, seed, uid, k, p, 1u, NULL);
        U_out[i] = a - b;
    }
    free(g.inv);
}

/* Q_k from given U values with the exact-sum convention: used by tests. */
double pwo_q_from_u(int64_t R, const float* U)
{
    i128 S1 = 0;
    u128 S2 = 0;
    for (int64_t p = 0; p < R; p++) {
        S1 += fix54(U[p]);
        S2 += sqfix64(U[p]);
    }
    return probe_q(S1, S2, R);
}

/* ------------------------------------------------------------------------ */
/* Q_k for a list of probes (sampled checks at full size), threads over k    */
/* ------------------------------------------------------------------------ */
typedef struct {
    const graph_t* g;
    uint64_t seed;
    int32_t s, t, L;
    uint32_t uid;
    int64_t R, B, M;
    const uint32_t* ks;
    double* q;
    int64_t count;
    int64_t next;
    pthread_mutex_t mu;
} qpool_t;

static void* q_worker(void* arg)
{
    qpool_t* pl = (qpool_t*)arg;
    domain_t d = make_domain(pl->g->n);
    for (;;) {
        pthread_mutex_lock(&pl->mu);
        int64_t i = pl->next++;
        pthread_mutex_unlock(&pl->mu);
        if (i >= pl->count) break;
        uint32_t k = pl->ks[i];
        /* the walks of probe k are those of its walk-sharing group */
        uint32_t kw = (uint32_t)group_first((int64_t)k, pl->B, pl->M);
        probe_t pr;
        make_probe(pl->seed, pl->uid, k, pl->g->n, &pr);
        i128 S1 = 0;
        u128 S2 = 0;
        for (int64_t p = 0; p < pl->R; p++) {
            float a, b;
            walk_sums(pl->g, &d, &pr, 1, (uint32_t)pl->s, pl->L, pl->seed, pl->uid, kw, (uint32_t)p, 0u, &a);
            walk_sums(pl->g, &d, &pr, 1, (uint32_t)pl->t, pl->L, pl->seed, pl->uid, kw, (uint32_t)p, 1u, &b);
            float U = a - b;
            S1 += fix54(U);
            S2 += sqfix64(U);
        }
        pl->q[i] = probe_q(S1, S2, pl->R);
    }
    return NULL;
}

int pwo_probe_q(uint32_t n, const int64_t* row_ptr, const int32_t* col, int32_t s, int32_t t,
                int32_t L, uint32_t uid, int64_t R, int64_t B, int64_t M, uint64_t seed, int64_t count,
                const uint32_t* ks, int nthreads, double* q_out)
{
    graph_t g = {n, row_ptr, col, NULL};
    g.inv = (float*)malloc(sizeof(float) * n);
    for (uint32_t v = 0; v < n; v++) g.inv[v] = 1.0f / (float)(row_ptr[v + 1] - row_ptr[v]);
    if (B < 1) B = 1;
    if (M < 1) M = 1;
    qpool_t pl = {&g, seed, s, t, L, uid, R, B, M, ks, q_out, count, 0, PTHREAD_MUTEX_INITIALIZER};
    if (nthreads < 1) nthreads = 1;
    if (nthreads > count) nthreads = (int)(count > 0 ? count : 1);
    pthread_t* th = (pthread_t*)malloc(sizeof(pthread_t) * (size_t)nthreads);
    for (int i = 0; i < nthreads; i++) pthread_create(&th[i], NULL, q_worker, &pl);
    for (int i = 0; i < nthreads; i++) pthread_join(th[i], NULL);
    free(th);
    free(g.inv);
    return 0;
}
