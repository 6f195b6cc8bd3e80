/*
 * Plain C replay of the Gibbs chains over Feynman paths (test
 * infrastructure only; shares nothing with the HIP path).
 *
 * Follows Fig. 2 of the paper, steps 1-3, with the sampling law of
 * Eq. (weightedS) (p_C proportional to |psi_C| = exp(-Re E)):
 *   step 1/2  each free p-bit is redrawn from its exact conditional
 *             (heat bath / Glauber: no rejection), colour by colour;
 *   step 3    after each post-burn-in sweep the path's output state alpha
 *             and phase exp(-i Im E) = exp(2 pi i k / 2^K) are binned,
 *             unless the path meets a soft zero (a zero entry replaced by
 *             e^(-J) for sampling, Appendix): then it is not a path of the
 *             circuit and is not binned.
 *
 * The conditional of free bit b is evaluated directly on the lattice:
 *   w_v = product over its real-energy factors (ascending gate order) of
 *         |U_g| at the lattice with bit b set to v (its cone toggled),
 *   P   = w_1 / (w_0 + w_1),   T = min(floor(P 2^32), 2^32 - 1),
 *   new = (u < T),  u = the Philox4x32-10 draw of this update.
 * The phase is the sum over all gates of their phase-table entries; the
 * output state is the last layer of the lattice.  Random numbers come from
 * Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11), counter
 * (sweep, b / 4, chain, circuit_id | tag << 16), key (seed lo, seed hi),
 * word b % 4.
 *
 * Built with: gcc -O2 -ffp-contract=off -shared -fPIC -pthread
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ---------------------------------------------------------------------- */
/* Philox4x32-10 from its published definition                            */
/* ---------------------------------------------------------------------- */
#define PHILOX_M0 0xD2511F53u
#define PHILOX_M1 0xCD9E8D57u
#define PHILOX_W0 0x9E3779B9u
#define PHILOX_W1 0xBB67AE85u

void oracle_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2],
                          uint32_t out[4]) {
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int r = 0; r < 10; ++r) {
        uint64_t p0 = (uint64_t)PHILOX_M0 * (uint64_t)c0;
        uint64_t p1 = (uint64_t)PHILOX_M1 * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += PHILOX_W0;
        k1 += PHILOX_W1;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* ---------------------------------------------------------------------- */
/* chain replay                                                            */
/* ---------------------------------------------------------------------- */
typedef struct {
    /* lattice */
    int n, d, K, L, W, h;
    const uint32_t *const_words; /* W */
    const int32_t *free_pos;     /* h */
    const uint32_t *cone;        /* h * W */
    /* gates */
    int G;
    const int32_t *arity;    /* G */
    const int32_t *in_bits;  /* G * 2 */
    const int32_t *out_bits; /* G * 2 */
    const double *mag;       /* G * 16, index out * 2^a + in */
    const int32_t *ph;       /* G * 16 */
    /* conditionals */
    const int32_t *factor_off; /* h + 1 */
    const int32_t *factor_ids;
    const int32_t *order; /* h: colour ascending, then b ascending */
    /* run */
    uint64_t seed;
    uint32_t circuit_id, tag;
    uint32_t chain_begin, chain_count;
    uint32_t sweep_offset, burn_in, sweeps;
    const uint32_t *init_state; /* chain_count * W or NULL */
    uint32_t *out_state;        /* chain_count * W or NULL */
    uint64_t *hist;             /* 2^(n+K) */
} oracle_run;

static inline int getbit(const uint32_t *x, int p) { return (x[p >> 5] >> (p & 31)) & 1u; }

static int gate_index(const oracle_run *R, int g, const uint32_t *x) {
    int a = R->arity[g], i = 0, o = 0;
    for (int j = 0; j < a; ++j) {
        i |= getbit(x, R->in_bits[2 * g + j]) << j;
        o |= getbit(x, R->out_bits[2 * g + j]) << j;
    }
    return o * (1 << a) + i;
}

static uint32_t threshold(const oracle_run *R, int b, const uint32_t *x, uint32_t *tmp) {
    int f0 = R->factor_off[b], f1 = R->factor_off[b + 1];
    if (f0 == f1) {
        /* no real-energy factor: w_0 = w_1 = 1, P = 1/2 */
        double P = 1.0 / (1.0 + 1.0);
        double t = floor(P * 4294967296.0);
        return (uint32_t)t;
    }
    int cur = getbit(x, R->free_pos[b]);
    double w[2];
    for (int v = 0; v < 2; ++v) {
        memcpy(tmp, x, sizeof(uint32_t) * R->W);
        if (cur != v)
            for (int k = 0; k < R->W; ++k) tmp[k] ^= R->cone[(size_t)b * R->W + k];
        double p = 1.0;
        for (int f = f0; f < f1; ++f) {
            int g = R->factor_ids[f];
            p = p * R->mag[16 * g + gate_index(R, g, tmp)];
        }
        w[v] = p;
    }
    double P = w[1] / (w[0] + w[1]);
    double t = floor(P * 4294967296.0);
    if (t > 4294967295.0) t = 4294967295.0;
    return (uint32_t)t;
}

static void sample(const oracle_run *R, const uint32_t *x, uint64_t *hist) {
    int n = R->n, d = R->d, K = R->K;
    uint32_t alpha = 0;
    for (int q = 0; q < n; ++q) alpha |= (uint32_t)getbit(x, d * n + q) << q;
    int64_t k = 0;
    for (int g = 0; g < R->G; ++g) {
        const int e = R->ph[16 * g + gate_index(R, g, x)];
        if (e < 0) return; /* a soft zero: not a path of the circuit, not binned */
        k += e;
    }
    uint32_t phi = (uint32_t)(k & ((1 << K) - 1));
    hist[((uint64_t)alpha << K) | phi] += 1;
}

/* The conditional threshold of free bit b at lattice x (as used above). */
uint32_t oracle_threshold(const oracle_run *R, int b, const uint32_t *x) {
    uint32_t *tmp = (uint32_t *)malloc(sizeof(uint32_t) * R->W);
    uint32_t t = threshold(R, b, x, tmp);
    free(tmp);
    return t;
}

typedef struct {
    const oracle_run *R;
    uint32_t c0, c1; /* local chain range */
    uint64_t *hist;
} job;

static void *worker(void *arg) {
    job *J = (job *)arg;
    const oracle_run *R = J->R;
    int W = R->W;
    uint32_t *x = (uint32_t *)malloc(sizeof(uint32_t) * W);
    uint32_t *tmp = (uint32_t *)malloc(sizeof(uint32_t) * W);
    uint32_t key[2] = {(uint32_t)R->seed, (uint32_t)(R->seed >> 32)};
    for (uint32_t lc = J->c0; lc < J->c1; ++lc) {
        uint32_t chain = R->chain_begin + lc;
        if (R->init_state)
            memcpy(x, R->init_state + (size_t)lc * W, sizeof(uint32_t) * W);
        else
            memcpy(x, R->const_words, sizeof(uint32_t) * W);
        uint32_t total = R->burn_in + R->sweeps;
        for (uint32_t it = 0; it < total; ++it) {
            uint32_t s = R->sweep_offset + it;
            for (int oi = 0; oi < R->h; ++oi) {
                int b = R->order[oi];
                uint32_t ctr[4] = {s, (uint32_t)(b >> 2), chain,
                                   R->circuit_id | (R->tag << 16)};
                uint32_t u4[4];
                oracle_philox4x32_10(ctr, key, u4);
                uint32_t u = u4[b & 3];
                uint32_t T = threshold(R, b, x, tmp);
                int nv = u < T;
                if (nv != getbit(x, R->free_pos[b]))
                    for (int k = 0; k < W; ++k) x[k] ^= R->cone[(size_t)b * W + k];
            }
            if (it >= R->burn_in) sample(R, x, J->hist);
        }
        if (R->out_state) memcpy(R->out_state + (size_t)lc * W, x, sizeof(uint32_t) * W);
    }
    free(x);
    free(tmp);
    return NULL;
}

/* Runs chain_count chains on `threads` POSIX threads; adds into R->hist. */
int oracle_gibbs_run(const oracle_run *R, int threads) {
    if (threads < 1) threads = 1;
    if ((uint32_t)threads > R->chain_count) threads = R->chain_count ? (int)R->chain_count : 1;
    size_t nb = (size_t)1 << (R->n + R->K);
    pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * threads);
    job *jobs = (job *)malloc(sizeof(job) * threads);
    for (int t = 0; t < threads; ++t) {
        jobs[t].R = R;
        jobs[t].c0 = (uint32_t)((uint64_t)R->chain_count * t / threads);
        jobs[t].c1 = (uint32_t)((uint64_t)R->chain_count * (t + 1) / threads);
        jobs[t].hist = (uint64_t *)calloc(nb, sizeof(uint64_t));
        if (!jobs[t].hist) return -1;
        pthread_create(&th[t], NULL, worker, &jobs[t]);
    }
    for (int t = 0; t < threads; ++t) {
        pthread_join(th[t], NULL);
        for (size_t i = 0; i < nb; ++i) R->hist[i] += jobs[t].hist[i];
        free(jobs[t].hist);
    }
    free(th);
    free(jobs);
    return 0;
}
