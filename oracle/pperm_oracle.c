/*
 * pperm_oracle.c -- plain CPU oracle for parallel flatPERM on Z^2 and Z^3.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct reference
 * that the GPU path is checked against.  Only the test-suite, the smoke check and
 * the CPU-baseline leg of the benchmark may load it.  It shares no source, header,
 * table or helper with the HIP library, and it never reads anything the GPU wrote.
 *
 * What it follows (Campbell & Janse van Rensburg, "Parallel PERM"):
 *   - Sec. 1: Rosenbluth growth.  a_+(w_n) counts the free edges at the endpoint,
 *     one of them is chosen uniformly, a_+(empty walk) = 2d; the chain probability
 *     is eqn (1), the Rosenbluth weight W = prod a_+ is eqn (2), and a trapped walk
 *     (a_+ = 0) ends its chain.  The sample average <W_n>_M = sum W_n / M of
 *     eqn (4) estimates c_n, where M counts passes through the empty walk.
 *   - Sec. 2: flatPERM.  r = W / [W_k] with the current weight included in the
 *     running average (eqn (6)); r >= 1 enriches into c copies (c = floor r with
 *     probability ceil r - r, else ceil r), each of weight W/c, grown on
 *     independently; r < 1 prunes with probability 1 - r, a survivor's weight is
 *     multiplied by 1/r.
 *   - Sec. 3 and Fig. 1: Algorithm 2 -- N sequences pool their weights in one
 *     shared W; M is the total number of passes of all sequences through the
 *     empty walk.  Algorithm 1 -- N independent sequences, averaged afterwards
 *     (eqn (7)).
 *
 * Readings taken where the paper is silent (each one is stated again in the
 * design notes of the repository):
 *   R1  sharing is epoch-synchronous: inside an epoch a sequence sees the pooled
 *       sums frozen at the last merge plus its own sums of the current epoch;
 *   R2  inside an epoch a sequence extrapolates the pool's progress from its own:
 *       est = (G_n + N * L_n) / (M_G + N * m) in Algorithm 2 (N sequences, L_n
 *       and m its own sums and tours of the epoch, its current weight and tour
 *       included), est = (G_n + L_n) / (M_G + m) with its own G, M_G in
 *       Algorithm 1; N = 1 is plain flatPERM's running average;
 *   R3  copies are grown depth first, copy 1 first, the rest from a LIFO stack;
 *   R4  r = W / est is evaluated as (W * M') / S for est = S / M' (S the weight
 *       sum, M' the tour count of R2), and a pruned-but-surviving walk takes
 *       weight est = S / M' (= W / r mathematically);
 *   R5  no control at n = 0, at n = n_max, or for a trapped walk; a resumed copy
 *       grows without a new control decision (the copies share one record);
 *   R6  randomness: Philox4x32-10, key = seed, counter = (k_lo, k_hi, t_lo, s),
 *       one block per growth event, k counted per tour in DFS order;
 *   R7  j-th free neighbour with j = (B0 * a_+) >> 32, neighbours in the order
 *       +x, -x, +y, -y, +z, -z; u = ((B1 >> 5) * 2^26 + (B2 >> 6)) * 2^-53;
 *       c = floor r iff (r not integral and u < (floor r + 1) - r); survive iff u < r;
 *   R8  weights and weight sums are extended-range numbers m * 2^e (FP64
 *       mantissa, int32 exponent) whose operations are correctly rounded; the
 *       weights of the first walks into new lengths shrink by a factor of about
 *       m per length and leave the FP64 range long before n = 500;
 *   R9  the pooled sums are merged with an aligned pairwise tree over sequences,
 *       padded with +0.0 to a power of two.
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -shared -fPIC (no -ffast-math).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror & Shaw, "Parallel random numbers: as  */
/* easy as 1, 2, 3", SC'11).  Ten rounds; each round multiplies words 0 and   */
/* 2 by the two Philox constants, swaps and xors with the round key; the key  */
/* is bumped by the Weyl constants between rounds.                            */
/* ------------------------------------------------------------------------ */
#define ORC_PHILOX_M0 0xD2511F53u
#define ORC_PHILOX_M1 0xCD9E8D57u
#define ORC_PHILOX_W0 0x9E3779B9u
#define ORC_PHILOX_W1 0xBB67AE85u

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t p0 = (uint64_t)ORC_PHILOX_M0 * (uint64_t)c0;
        uint64_t p1 = (uint64_t)ORC_PHILOX_M1 * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += ORC_PHILOX_W0;
        k1 += ORC_PHILOX_W1;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* ------------------------------------------------------------------------ */
/* Extended-range weights (reading R8).  A weight is x = m * 2^e with the   */
/* FP64 mantissa m in [0.5, 1) (m = 0, e = 0 for zero) and an int32          */
/* exponent e.  Each operation below is the correctly rounded IEEE result of */
/* the exact operation on the represented values, renormalised exactly:      */
/* nothing can underflow or overflow, and no transcendental function is      */
/* ever used on the decision path.                                           */
/* ------------------------------------------------------------------------ */
typedef struct { double m; int32_t e; uint32_t pad; } orc_xf;

static orc_xf orc_xf_norm(double x, int32_t e)
{
    orc_xf r;
    int k = 0;
    double m = frexp(x, &k);
    if (m == 0.0) { r.m = 0.0; r.e = 0; r.pad = 0; return r; }
    r.m = m; r.e = e + k; r.pad = 0;
    return r;
}

static orc_xf orc_xf_from_double(double x) { return orc_xf_norm(x, 0); }

/* a + b: the operand with the larger exponent keeps its scale and the other is
 * shifted onto it (an exact scaling by a power of two); beyond 63 binades the
 * smaller operand cannot change the rounded sum and is dropped. */
orc_xf orc_xf_add(orc_xf a, orc_xf b)
{
    if (a.m == 0.0) return b;
    if (b.m == 0.0) return a;
    if (a.e < b.e) { orc_xf t = a; a = b; b = t; }
    int64_t d = (int64_t)a.e - (int64_t)b.e;
    if (d > 63) return a;
    return orc_xf_norm(a.m + ldexp(b.m, (int)(-d)), a.e);
}

/* a * k and a / k for a positive integer-valued double k. */
orc_xf orc_xf_mul(orc_xf a, double k) { return orc_xf_norm(a.m * k, a.e); }
orc_xf orc_xf_div(orc_xf a, double k) { return orc_xf_norm(a.m / k, a.e); }

/* a / b as an ordinary double (b != 0): ldexp(a.m / b.m, a.e - b.e), with the
 * exponent difference clamped to [-1000, 1000] (0 below, 2^1000 above). */
double orc_xf_ratio(orc_xf a, orc_xf b)
{
    if (a.m == 0.0) return 0.0;
    int64_t d = (int64_t)a.e - (int64_t)b.e;
    if (d < -1000) return 0.0;
    if (d > 1000) return ldexp(1.0, 1000);
    return ldexp(a.m / b.m, (int)d);
}

/* Test hooks: the operations on arrays (op 0 add, 1 mul, 2 div). */
void orc_xf_apply(int op, const double* am, const int32_t* ae, const double* bm, const int32_t* be,
                  const double* k, int64_t n, double* om, int32_t* oe)
{
    for (int64_t i = 0; i < n; ++i) {
        orc_xf a = { am[i], ae[i], 0 }, r;
        if (op == 0) { orc_xf b = { bm[i], be[i], 0 }; r = orc_xf_add(a, b); }
        else if (op == 1) r = orc_xf_mul(a, k[i]);
        else r = orc_xf_div(a, k[i]);
        om[i] = r.m; oe[i] = r.e;
    }
}

void orc_xf_normalize(const double* x, int64_t n, double* om, int32_t* oe)
{
    for (int64_t i = 0; i < n; ++i) { orc_xf r = orc_xf_from_double(x[i]); om[i] = r.m; oe[i] = r.e; }
}

/* ------------------------------------------------------------------------ */
/* Occupancy set: open addressing, linear probing, backward-shift deletion   */
/* (Knuth, TAOCP vol. 3, 6.4, Algorithm R).  Keys are packed coordinates      */
/* with 21 bits per axis; key 0 never occurs because the offset is 2^20.     */
/* ------------------------------------------------------------------------ */
typedef struct {
    uint64_t* slot;
    uint64_t mask;
    uint64_t count;
} orc_set;

static uint64_t orc_key(int x, int y, int z)
{
    return ((uint64_t)(uint32_t)(x + (1 << 20)))
         | ((uint64_t)(uint32_t)(y + (1 << 20)) << 21)
         | ((uint64_t)(uint32_t)(z + (1 << 20)) << 42);
}

static uint64_t orc_mix(uint64_t k)
{
    /* splitmix64 finaliser */
    k ^= k >> 30; k *= 0xBF58476D1CE4E5B9ull;
    k ^= k >> 27; k *= 0x94D049BB133111EBull;
    k ^= k >> 31;
    return k;
}

static int orc_set_init(orc_set* s, uint64_t max_items)
{
    uint64_t cap = 16;
    while (cap < 4 * (max_items + 1)) cap <<= 1;
    s->slot = (uint64_t*)calloc(cap, sizeof(uint64_t));
    s->mask = cap - 1;
    s->count = 0;
    return s->slot ? 0 : -1;
}

static void orc_set_free(orc_set* s) { free(s->slot); s->slot = NULL; }

static int orc_set_contains(const orc_set* s, uint64_t key)
{
    uint64_t i = orc_mix(key) & s->mask;
    for (;;) {
        if (s->slot[i] == 0) return 0;
        if (s->slot[i] == key) return 1;
        i = (i + 1) & s->mask;
    }
}

static void orc_set_insert(orc_set* s, uint64_t key)
{
    uint64_t i = orc_mix(key) & s->mask;
    while (s->slot[i] != 0) {
        if (s->slot[i] == key) return;
        i = (i + 1) & s->mask;
    }
    s->slot[i] = key;
    s->count++;
}

static void orc_set_remove(orc_set* s, uint64_t key)
{
    uint64_t i = orc_mix(key) & s->mask;
    while (s->slot[i] != key) {
        if (s->slot[i] == 0) return;
        i = (i + 1) & s->mask;
    }
    /* Algorithm R: close the hole by shifting back later members of the run. */
    uint64_t j = i;
    for (;;) {
        s->slot[i] = 0;
        for (;;) {
            j = (j + 1) & s->mask;
            if (s->slot[j] == 0) { s->count--; return; }
            uint64_t home = orc_mix(s->slot[j]) & s->mask;
            /* the entry at j may move to i iff home lies cyclically outside (i, j] */
            int stays = (i <= j) ? (i < home && home <= j) : (i < home || home <= j);
            if (!stays) break;
        }
        s->slot[i] = s->slot[j];
        i = j;
    }
}

/* Exposed for the set's own unit test: op 0 = insert, 1 = remove, 2 = query;
 * writes query answers into out[] in order and returns the final count. */
int64_t orc_set_selftest(const int32_t* ops, const int32_t* xyz, int64_t n_ops,
                         int32_t* out, int64_t max_items)
{
    orc_set s;
    if (orc_set_init(&s, (uint64_t)max_items)) return -1;
    int64_t q = 0;
    for (int64_t i = 0; i < n_ops; ++i) {
        uint64_t k = orc_key(xyz[3 * i], xyz[3 * i + 1], xyz[3 * i + 2]);
        if (ops[i] == 0) orc_set_insert(&s, k);
        else if (ops[i] == 1) orc_set_remove(&s, k);
        else out[q++] = orc_set_contains(&s, k);
    }
    int64_t c = (int64_t)s.count;
    orc_set_free(&s);
    return c;
}

/* ------------------------------------------------------------------------ */
/* Walk state and the free-neighbour scan (a_+ of Sec. 1).                   */
/* ------------------------------------------------------------------------ */
static const int ORC_DX[6] = { 1, -1, 0,  0, 0,  0 };
static const int ORC_DY[6] = { 0,  0, 1, -1, 0,  0 };
static const int ORC_DZ[6] = { 0,  0, 0,  0, 1, -1 };

typedef struct {
    int dim;
    int64_t n;          /* current length */
    int32_t* x; int32_t* y; int32_t* z;   /* sites 0..n */
    orc_set occ;
} orc_walk;

static int orc_walk_init(orc_walk* w, int dim, int64_t n_max)
{
    w->dim = dim;
    w->n = 0;
    w->x = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n_max + 1));
    w->y = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n_max + 1));
    w->z = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n_max + 1));
    if (!w->x || !w->y || !w->z || orc_set_init(&w->occ, (uint64_t)n_max + 1)) return -1;
    w->x[0] = w->y[0] = w->z[0] = 0;
    orc_set_insert(&w->occ, orc_key(0, 0, 0));
    return 0;
}

static void orc_walk_free(orc_walk* w)
{
    free(w->x); free(w->y); free(w->z);
    orc_set_free(&w->occ);
}

/* Bit b of the result is set iff neighbour b of the endpoint is unoccupied;
 * *a receives the number of set bits, i.e. a_+(w_n). */
static unsigned orc_free_mask(const orc_walk* w, int* a)
{
    unsigned mask = 0;
    int cnt = 0;
    int64_t n = w->n;
    for (int b = 0; b < 2 * w->dim; ++b) {
        uint64_t k = orc_key(w->x[n] + ORC_DX[b], w->y[n] + ORC_DY[b], w->z[n] + ORC_DZ[b]);
        if (!orc_set_contains(&w->occ, k)) { mask |= 1u << b; ++cnt; }
    }
    *a = cnt;
    return mask;
}

static void orc_walk_push(orc_walk* w, int dir)
{
    int64_t n = w->n;
    w->x[n + 1] = w->x[n] + ORC_DX[dir];
    w->y[n + 1] = w->y[n] + ORC_DY[dir];
    w->z[n + 1] = w->z[n] + ORC_DZ[dir];
    orc_set_insert(&w->occ, orc_key(w->x[n + 1], w->y[n + 1], w->z[n + 1]));
    w->n = n + 1;
}

static void orc_walk_truncate(orc_walk* w, int64_t len)
{
    while (w->n > len) {
        int64_t n = w->n;
        orc_set_remove(&w->occ, orc_key(w->x[n], w->y[n], w->z[n]));
        w->n = n - 1;
    }
}

/* The j-th set bit (0-based, lowest first) of mask. */
static int orc_nth_free(unsigned mask, unsigned j)
{
    for (int b = 0; b < 6; ++b) {
        if (mask & (1u << b)) {
            if (j == 0) return b;
            --j;
        }
    }
    return -1;
}

/* ------------------------------------------------------------------------ */
/* Parameters, statistics and the RNG contract (readings R6, R7).            */
/* ------------------------------------------------------------------------ */
enum { ORC_MODE_SHARED = 0, ORC_MODE_INDEPENDENT = 1, ORC_MODE_ROSENBLUTH = 2 };

typedef struct {
    int32_t dim;
    int32_t mode;
    int64_t n_max;
    uint64_t seed;
    uint32_t stream;        /* xored into the key's high word (problem id) */
    uint32_t pad;
    uint64_t step_cap;      /* growth steps per sequence per call; 0 = none */
    uint64_t n_pool;        /* N of reading R2 (number of pooled sequences) */
} orc_params;

/* Per-sequence counters, cumulative over the whole run. */
typedef struct {
    uint64_t steps;      /* growth steps (walk-steps) */
    uint64_t events;     /* RNG blocks drawn */
    uint64_t enrich;     /* control decisions with c > 1 */
    uint64_t copies;     /* sum of (c - 1) */
    uint64_t prunes;     /* walks removed by pruning */
    uint64_t traps;      /* arrivals with a_+ = 0 */
    uint64_t tours;      /* passes through the empty walk */
    uint64_t max_depth;  /* deepest copy stack */
    uint64_t digest;     /* FNV-1a 32 over one byte per growth, dir | a_+ << 3, zero-extended */
    uint64_t capped;     /* 1 once the step cap stopped this sequence */
} orc_seq_stats;

/* The trajectory digest is instrumentation for comparing walks, not part of
 * the method: FNV-1a with 32-bit state (offset basis and prime of its
 * published definition). */
#define ORC_FNV_OFFSET 2166136261u
#define ORC_FNV_PRIME  16777619u

void orc_stats_init(orc_seq_stats* st, int64_t count)
{
    memset(st, 0, sizeof(orc_seq_stats) * (size_t)count);
    for (int64_t i = 0; i < count; ++i) st[i].digest = ORC_FNV_OFFSET;
}

static void orc_draw(const orc_params* P, uint32_t s, uint64_t t, uint64_t k, uint32_t B[4])
{
    uint32_t ctr[4] = { (uint32_t)k, (uint32_t)(k >> 32), (uint32_t)t, s };
    uint32_t key[2] = { (uint32_t)P->seed, (uint32_t)(P->seed >> 32) ^ P->stream };
    orc_philox4x32_10(ctr, key, B);
}

static double orc_uniform53(const uint32_t B[4])
{
    double hi = (double)(B[1] >> 5);
    double lo = (double)(B[2] >> 6);
    return (hi * 67108864.0 + lo) * (1.0 / 9007199254740992.0);
}

/* ------------------------------------------------------------------------ */
/* One sequence, `tours` tours, against frozen pooled sums (readings R1-R5).  */
/*                                                                          */
/*   G, MG : the pooled sums this sequence sees (Alg 2: shared by all; Alg 1: */
/*           the sequence's own; unused for the Rosenbluth mode)             */
/*   L, H  : this sequence's sums of the current epoch (length n_max + 1)     */
/*   LR    : this sequence's sums of W * R^2 (squared end-to-end distance),   */
/*           the numerator of the ratio estimator, eqn (5); NULL: none     */
/*   m     : this sequence's tours in the current epoch                      */
/*   t     : this sequence's global tour counter                             */
/* Returns 0, or 1 if the step cap stopped the sequence.                    */
/* ------------------------------------------------------------------------ */
typedef struct { int64_t n; uint64_t remaining; orc_xf w; } orc_entry;

int orc_run_sequence(const orc_params* P, const orc_xf* G, uint64_t MG,
                     uint32_t s, uint64_t* t, uint32_t tours,
                     orc_xf* L, uint32_t* H, uint32_t* m, orc_seq_stats* st, orc_xf* LR)
{
    const int dim = P->dim;
    const int64_t n_max = P->n_max;
    const int control_allowed = (P->mode != ORC_MODE_ROSENBLUTH);
    /* reading R2: own epoch data stands for the whole pool's (N = 1 in Alg 1) */
    const double pool = (P->mode == ORC_MODE_SHARED) ? (double)P->n_pool : 1.0;
    const orc_xf one = orc_xf_from_double(1.0);
    orc_walk walk;
    orc_entry* stack = (orc_entry*)malloc(sizeof(orc_entry) * (size_t)(n_max + 1));
    if (!stack || orc_walk_init(&walk, dim, n_max)) { free(stack); return -1; }
    uint64_t steps_this_call = 0;
    int capped = 0;

    for (uint32_t tour = 0; tour < tours && !capped; ++tour) {
        /* Tour start: a pass through the empty walk (eqn (4), M). */
        uint64_t tt = *t;
        *t += 1;
        *m += 1;
        st->tours += 1;
        orc_walk_truncate(&walk, 0);
        int64_t depth = 0;
        uint64_t k = 0;
        orc_xf w = one;
        L[0] = orc_xf_add(L[0], w);      /* W_0 = 1 */
        H[0] += 1;
        int control = 0;    /* no decision at n = 0 */
        int a;
        unsigned mask = orc_free_mask(&walk, &a);   /* a = 2d */

        for (;;) {
            /* ---- growth event at length walk.n with weight w, a > 0 ---- */
            uint32_t B[4];
            orc_draw(P, s, tt, k, B);
            k += 1;
            st->events += 1;
            int pruned = 0;
            if (control) {
                int64_t n = walk.n;
                /* eqn (6): r = W / [W_n] with [W_n] = sum / tours_seen, evaluated
                 * as r = (W * tours_seen) / sum (one division) */
                orc_xf sum = orc_xf_add(G[n], orc_xf_mul(L[n], pool));
                double tours_seen = (double)(MG + (uint64_t)pool * (uint64_t)(*m));
                double r = orc_xf_ratio(orc_xf_mul(w, tours_seen), sum);
                double u = orc_uniform53(B);
                if (r >= 1.0) {
                    double f = floor(r);
                    double c;
                    if (r != f && u < (f + 1.0) - r) c = f;
                    else c = (r == f) ? f : f + 1.0;
                    w = orc_xf_div(w, c);
                    if (c > 1.0) {
                        stack[depth].n = n;
                        stack[depth].remaining = (uint64_t)c - 1;
                        stack[depth].w = w;
                        depth += 1;
                        if ((uint64_t)depth > st->max_depth) st->max_depth = (uint64_t)depth;
                        st->enrich += 1;
                        st->copies += (uint64_t)c - 1;
                    }
                } else {
                    /* survivor: W / r, which is the running average itself */
                    if (u < r) w = orc_xf_div(sum, tours_seen);
                    else { pruned = 1; st->prunes += 1; }
                }
            }

            int need_backtrack = pruned;
            if (!pruned) {
                /* Rosenbluth growth (Sec. 1): the j-th free neighbour, W *= a_+ (eqn (2)). */
                unsigned j = (unsigned)(((uint64_t)B[0] * (uint64_t)a) >> 32);
                int dir = orc_nth_free(mask, j);
                st->digest = (uint32_t)(((uint32_t)st->digest ^ (uint32_t)(dir | (a << 3))) * ORC_FNV_PRIME);
                w = orc_xf_mul(w, (double)a);
                orc_walk_push(&walk, dir);
                st->steps += 1;
                steps_this_call += 1;
                /* arrival: record into the running sums (eqn (4)) */
                L[walk.n] = orc_xf_add(L[walk.n], w);
                H[walk.n] += 1;
                if (LR) {
                    const int64_t q = walk.n;
                    const double r2 = (double)((int64_t)walk.x[q] * walk.x[q] + (int64_t)walk.y[q] * walk.y[q] +
                                               (int64_t)walk.z[q] * walk.z[q]);
                    LR[q] = orc_xf_add(LR[q], orc_xf_mul(w, r2));
                }
                if (P->step_cap && steps_this_call >= P->step_cap) { capped = 1; break; }
                if (walk.n == n_max) {
                    need_backtrack = 1;
                } else {
                    mask = orc_free_mask(&walk, &a);
                    if (a == 0) { need_backtrack = 1; st->traps += 1; }
                    else control = control_allowed;
                }
            }

            if (need_backtrack) {
                /* resume the most recent pending copy, or end the tour */
                if (depth == 0) break;
                orc_entry* top = &stack[depth - 1];
                int64_t rn = top->n;
                w = top->w;
                top->remaining -= 1;
                if (top->remaining == 0) depth -= 1;
                orc_walk_truncate(&walk, rn);
                mask = orc_free_mask(&walk, &a);
                control = 0;   /* the copies share the record made at rn */
            }
        }
    }
    if (capped) st->capped = 1;
    orc_walk_free(&walk);
    free(stack);
    return capped;
}

/* ------------------------------------------------------------------------ */
/* One epoch over all sequences.  Sequences do not interact inside an epoch  */
/* (reading R1), so they may run on any number of host threads; the result   */
/* does not depend on the thread count.                                      */
/*                                                                          */
/* Shared mode: G[n1], MG[1].  Independent mode: G[N][n1], MG[N].            */
/* L[N][n1], H[N][n1], m[N], t[N], stats[N].                                 */
/* ids == NULL runs every sequence 0..N-1; otherwise only ids[0..n_ids-1].   */
/* ------------------------------------------------------------------------ */
int orc_run_epoch(const orc_params* P, int64_t N, const orc_xf* G, const uint64_t* MG,
                  uint64_t* t, uint32_t tours, orc_xf* L, uint32_t* H, uint32_t* m,
                  orc_seq_stats* stats, const int64_t* ids, int64_t n_ids, int threads, orc_xf* LR)
{
    const int64_t n1 = P->n_max + 1;
    const int64_t count = ids ? n_ids : N;
    int any_capped = 0;
    orc_params Q = *P;
    Q.n_pool = (uint64_t)N;
#ifdef _OPENMP
    if (threads <= 0) threads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 1) num_threads(threads) reduction(|:any_capped)
#endif
    for (int64_t i = 0; i < count; ++i) {
        const int64_t s = ids ? ids[i] : i;
        const orc_xf* Gs = G;
        uint64_t Ms = MG ? MG[0] : 0;
        if (P->mode == ORC_MODE_INDEPENDENT) { Gs = G + s * n1; Ms = MG[s]; }
        int rc = orc_run_sequence(&Q, Gs, Ms, (uint32_t)s, &t[s], tours,
                                  L + s * n1, H + s * n1, &m[s], &stats[s], LR ? LR + s * n1 : NULL);
        if (rc != 0) any_capped |= 1;
    }
    (void)threads;
    return any_capped;
}

/* ------------------------------------------------------------------------ */
/* Merge (reading R9): the aligned pairwise tree over sequences.             */
/* ------------------------------------------------------------------------ */
static orc_xf orc_pairwise(const orc_xf* L, int64_t n1, int64_t n, int64_t N,
                           int64_t lo, int64_t len)
{
    if (len == 1) {
        if (lo < N) return L[lo * n1 + n];
        orc_xf z = { 0.0, 0, 0 };
        return z;
    }
    int64_t half = len / 2;
    orc_xf left = orc_pairwise(L, n1, n, N, lo, half);
    orc_xf right = orc_pairwise(L, n1, n, N, lo + half, half);
    return orc_xf_add(left, right);
}

/* Shared mode: G[n] += tree(L[.][n]); HG[n] += sum H[.][n]; MG += sum m.
 * Independent mode: per sequence, G[s][n] += L[s][n] (and the same for HG, MG).
 * Afterwards L, H and m are zero. */
void orc_merge(const orc_params* P, int64_t N, orc_xf* L, uint32_t* H, uint32_t* m,
               orc_xf* G, uint64_t* HG, uint64_t* MG, orc_xf* LR, orc_xf* GR)
{
    const int64_t n1 = P->n_max + 1;
    if (P->mode == ORC_MODE_INDEPENDENT) {
        for (int64_t s = 0; s < N; ++s) {
            for (int64_t n = 0; n < n1; ++n) {
                G[s * n1 + n] = orc_xf_add(G[s * n1 + n], L[s * n1 + n]);
                HG[s * n1 + n] += H[s * n1 + n];
            }
            MG[s] += m[s];
        }
    } else {
        int64_t P2 = 1;
        while (P2 < N) P2 <<= 1;
        for (int64_t n = 0; n < n1; ++n) {
            G[n] = orc_xf_add(G[n], orc_pairwise(L, n1, n, N, 0, P2));
            if (LR && GR) GR[n] = orc_xf_add(GR[n], orc_pairwise(LR, n1, n, N, 0, P2));
            uint64_t h = 0;
            for (int64_t s = 0; s < N; ++s) h += H[s * n1 + n];
            HG[n] += h;
        }
        uint64_t mm = 0;
        for (int64_t s = 0; s < N; ++s) mm += m[s];
        MG[0] += mm;
    }
    memset(L, 0, sizeof(orc_xf) * (size_t)(N * n1));
    if (LR) memset(LR, 0, sizeof(orc_xf) * (size_t)(N * n1));
    memset(H, 0, sizeof(uint32_t) * (size_t)(N * n1));
    memset(m, 0, sizeof(uint32_t) * (size_t)N);
}

/* Group sums for the relative-error estimate of c_{n_max}: sequences fall in
 * 16 groups by s mod 16.  Group k adds, from zero and in increasing s, the
 * weights its sequences recorded at n_max in the open epoch, then adds that to
 * its running total; its tour count grows by its sequences' m.  Called before
 * orc_merge (which zeroes L and m). */
void orc_group_sums(const orc_params* P, int64_t N, const orc_xf* L, const uint32_t* m,
                    orc_xf* gsum, uint64_t* gtours)
{
    const int64_t n1 = P->n_max + 1;
    for (int64_t k = 0; k < 16; ++k) {
        orc_xf acc = { 0.0, 0, 0 };
        uint64_t tours = 0;
        for (int64_t s = k; s < N; s += 16) {
            acc = orc_xf_add(acc, L[s * n1 + P->n_max]);
            tours += m[s];
        }
        gsum[k] = orc_xf_add(gsum[k], acc);
        gtours[k] += tours;
    }
}

/* Ratio estimator (eqn (5)) of the mean squared end-to-end distance:
 * <R^2>_n = (sum of W R^2) / (sum of W) at each length, NaN where no sample. */
void orc_observable_r2(int64_t n_max, const orc_xf* G, const orc_xf* GR, double* out)
{
    for (int64_t n = 0; n <= n_max; ++n)
        out[n] = (G[n].m == 0.0) ? NAN : ldexp(GR[n].m / G[n].m, GR[n].e - G[n].e);
}

/* Estimates (eqn (4)): log c_n = ln G_n.m + G_n.e ln 2 - ln M. */
void orc_log_estimates(int64_t n_max, const orc_xf* G, uint64_t MG, double* out)
{
    for (int64_t n = 0; n <= n_max; ++n) {
        out[n] = log(G[n].m) + (double)G[n].e * 0.69314718055994530942 - log((double)MG);
    }
}

/* ------------------------------------------------------------------------ */
/* Plain flatPERM written recursively in the order Sec. 2 describes it: the  */
/* arrival records, the decision makes c copies, each copy grows on.  Used  */
/* only as a cross-check of the iterative form above (one sequence, one      */
/* epoch).  The state of the recursion lives in `orc_recur`.                 */
/* ------------------------------------------------------------------------ */
typedef struct {
    const orc_params* P;
    orc_walk walk;
    orc_xf* L; uint32_t* H;
    uint64_t m;        /* tours so far, including the current one */
    uint64_t t;        /* current tour index */
    uint64_t k;        /* events drawn in the current tour */
} orc_recur;

static void orc_rec_arrive(orc_recur* R, orc_xf w);

static void orc_rec_grow(orc_recur* R, orc_xf w, int control)
{
    const orc_params* P = R->P;
    uint32_t B[4];
    orc_draw(P, 0, R->t, R->k, B);
    R->k += 1;
    uint64_t c = 1;
    if (control) {
        int64_t n = R->walk.n;
        double r = orc_xf_ratio(orc_xf_mul(w, (double)R->m), R->L[n]);
        double u = orc_uniform53(B);
        if (r >= 1.0) {
            double f = floor(r);
            double cf = (r != f && u < (f + 1.0) - r) ? f : ceil(r);
            c = (uint64_t)cf;
            w = orc_xf_div(w, cf);
        } else if (u < r) {
            w = orc_xf_div(R->L[n], (double)R->m);
        } else {
            return;    /* pruned */
        }
    }
    /* copy 1 grows with this event's draw */
    int a;
    unsigned mask = orc_free_mask(&R->walk, &a);
    unsigned j = (unsigned)(((uint64_t)B[0] * (uint64_t)a) >> 32);
    int dir = orc_nth_free(mask, j);
    int64_t n = R->walk.n;
    orc_walk_push(&R->walk, dir);
    orc_rec_arrive(R, orc_xf_mul(w, (double)a));
    orc_walk_truncate(&R->walk, n);
    /* copies 2..c grow independently, each from a fresh event */
    for (uint64_t i = 1; i < c; ++i) orc_rec_grow(R, w, 0);
}

static void orc_rec_arrive(orc_recur* R, orc_xf w)
{
    int64_t n = R->walk.n;
    R->L[n] = orc_xf_add(R->L[n], w);
    R->H[n] += 1;
    if (n == R->P->n_max) return;
    int a;
    orc_free_mask(&R->walk, &a);
    if (a == 0) return;
    orc_rec_grow(R, w, R->P->mode != ORC_MODE_ROSENBLUTH);
}

int orc_plain_recursive(const orc_params* P, uint32_t tours, orc_xf* L, uint32_t* H)
{
    orc_recur R;
    R.P = P; R.L = L; R.H = H; R.m = 0; R.t = 0; R.k = 0;
    if (orc_walk_init(&R.walk, P->dim, P->n_max)) return -1;
    const orc_xf one = orc_xf_from_double(1.0);
    for (uint32_t i = 0; i < tours; ++i) {
        R.m += 1;
        R.t = i;
        R.k = 0;
        L[0] = orc_xf_add(L[0], one);
        H[0] += 1;
        orc_rec_grow(&R, one, 0);
    }
    orc_walk_free(&R.walk);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Forced-choice drive of the step functions above: every chain of every    */
/* length <= n_max is grown once, through the same free-neighbour scan and   */
/* the same weight update the sampler uses.                                  */
/*   count[n]   : number of chains of length n reached (must be c_n)         */
/*   bad[0]     : chains whose weight differs from prod a_+                  */
/* The product prod a_+ is carried here as an exact integer, independently   */
/* of the floating-point update, so this checks eqns (1)-(3) chain by chain. */
/* ------------------------------------------------------------------------ */
static void orc_force_rec(orc_walk* W, int64_t n_max, orc_xf w, uint64_t prod,
                          uint64_t* count, uint64_t* bad, uint64_t* r2sum)
{
    int64_t n = W->n;
    count[n] += 1;
    r2sum[n] += (uint64_t)((int64_t)W->x[n] * W->x[n] + (int64_t)W->y[n] * W->y[n] + (int64_t)W->z[n] * W->z[n]);
    if (ldexp(w.m, w.e) != (double)prod) bad[0] += 1;
    if (n == n_max) return;
    int a;
    unsigned mask = orc_free_mask(W, &a);
    for (int j = 0; j < a; ++j) {
        int dir = orc_nth_free(mask, (unsigned)j);
        orc_xf w2 = orc_xf_mul(w, (double)a);
        orc_walk_push(W, dir);
        orc_force_rec(W, n_max, w2, prod * (uint64_t)a, count, bad, r2sum);
        orc_walk_truncate(W, n);
    }
}

int orc_forced_enumerate(int dim, int64_t n_max, uint64_t* count, uint64_t* bad, uint64_t* r2sum)
{
    orc_walk W;
    if (orc_walk_init(&W, dim, n_max)) return -1;
    memset(count, 0, sizeof(uint64_t) * (size_t)(n_max + 1));
    memset(r2sum, 0, sizeof(uint64_t) * (size_t)(n_max + 1));
    bad[0] = 0;
    orc_force_rec(&W, n_max, orc_xf_from_double(1.0), 1, count, bad, r2sum);
    orc_walk_free(&W);
    return 0;
}
