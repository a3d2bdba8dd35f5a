/*
 * paper_mt.c -- CPU BASELINE, TEST INFRASTRUCTURE ONLY.
 *
 * The paper's own multithreaded CPU design of the cipher (Sec. 2,
 * Algorithms 1 and 2; the speed evaluation of Sec. 3), used to time the
 * paper's design on the host of the GPU machine and checked against the
 * single-threaded oracle.  It reuses the oracle's pinned primitives (the
 * PLCM byte generator of Eq. (5), the band bounds and the shift table of
 * Eq. (1)) and shares nothing with the GPU library.
 *
 * One POSIX thread per subframe, as in the paper.  For every frame each
 * thread
 *   1. draws its subframe's r*S_i keystream bytes from its own pair of
 *      PLCMs (Algorithm 2, "Iterate PRBG_a^i ... byte sequence B_i");
 *   2. computes the row shifts g of Eq. (1) for the frame (every thread keeps
 *      its own table, so no thread waits for another here);
 *   3. for each of the r rounds: confuses the pixels of its subframe -- each
 *      source pixel (a, o) of its rows is written to (alpha, beta) of the
 *      shared confused frame --, waits at a barrier, diffuses its subframe
 *      (Eq. 3) seeded with the last byte of the next subframe of the confused
 *      frame, and waits at a second barrier.
 * That is 2r barriers per frame.  The readings are the oracle's (band
 * bounds, HWC pixels moving whole, the seed rule, keystream layout).
 */
#define _POSIX_C_SOURCE 200809L  /* pthread barriers under -std=c11 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

uint32_t oracle_band_lo(uint32_t H, uint32_t n, uint32_t i);
void oracle_gtable(uint32_t H, uint32_t s_c, int64_t *g);
void oracle_plcm_bytes(double *x1, double p1, double *x2, double p2, uint64_t nbytes,
                       uint8_t *out);

typedef struct {
    uint32_t H, W, C, n, r;
    const double *pm;     /* n records (x0_1, p_1, x0_2, p_2); p used */
    double *state;        /* n pairs (x_1, x_2), advanced */
    const uint8_t *in;
    uint8_t *out;
    const uint32_t *s_c;
    uint64_t T;
    uint8_t *work;        /* round input/output between rounds (one frame) */
    uint8_t *conf;        /* confused frame of the current round */
    pthread_barrier_t bar;
} mt_job;

typedef struct {
    mt_job *job;
    uint32_t band;
} mt_arg;

static int64_t wrap(int64_t x, int64_t m)
{
    int64_t v = x % m;
    return v < 0 ? v + m : v;
}

static void *mt_worker(void *p)
{
    const mt_arg *arg = (const mt_arg *)p;
    mt_job *J = arg->job;
    const uint32_t i = arg->band, H = J->H, W = J->W, C = J->C, n = J->n, r = J->r;
    const uint64_t row = (uint64_t)W * C, F = (uint64_t)H * row;
    const uint32_t lo = oracle_band_lo(H, n, i), hi = oracle_band_lo(H, n, i + 1);
    const uint64_t S = (uint64_t)(hi - lo) * row;
    const uint32_t nb = (i + 1) % n;
    const uint64_t next_last = (uint64_t)oracle_band_lo(H, n, nb + 1) * row - 1;
    uint8_t *ks = (uint8_t *)malloc(r * S);
    int64_t *g = (int64_t *)malloc(sizeof(int64_t) * H);
    if (!ks || !g) abort();  /* tiny allocations; the caller sized the job */
    for (uint64_t t = 0; t < J->T; t++) {
        oracle_plcm_bytes(&J->state[2 * i], J->pm[4 * i + 1], &J->state[2 * i + 1],
                          J->pm[4 * i + 3], r * S, ks);
        oracle_gtable(H, J->s_c[t], g);
        for (uint32_t j = 0; j < r; j++) {
            const uint8_t *src = j == 0 ? J->in + t * F : J->work;
            uint8_t *dst = j + 1 == r ? J->out + t * F : J->work;
            /* confusion (Eq. 1) of the pixels of this subframe */
            for (uint32_t a = lo; a < hi; a++)
                for (uint32_t o = 0; o < W; o++) {
                    const int64_t alpha = wrap((int64_t)a + o, H);
                    const int64_t beta = wrap((int64_t)o + g[alpha], W);
                    memcpy(J->conf + ((uint64_t)alpha * W + beta) * C,
                           src + ((uint64_t)a * W + o) * C, C);
                }
            pthread_barrier_wait(&J->bar);
            /* diffusion (Eq. 3) of this subframe, round j's keystream bytes */
            const uint8_t *Y = J->conf + (uint64_t)lo * row;
            const uint8_t *b = ks + (uint64_t)j * S;
            uint8_t *Z = dst + (uint64_t)lo * row;
            uint8_t prev = J->conf[next_last];
            for (uint64_t k = 0; k < S; k++) {
                Z[k] = (uint8_t)(b[k] ^ (uint8_t)(Y[k] + b[k]) ^ prev);
                prev = Z[k];
            }
            pthread_barrier_wait(&J->bar);
        }
    }
    free(ks);
    free(g);
    return NULL;
}

/* Encrypt T frames (HWC, back to back) with the PLCM generators of the n
 * records in pm (x0_1, p_1, x0_2, p_2); state (2n doubles) holds the current
 * x of both maps of every band and is advanced.  Returns 0, or -1 if the
 * work buffers or threads could not be created. */
int paper_mt_encrypt(uint32_t H, uint32_t W, uint32_t C, uint32_t n, uint32_t r,
                     const double *pm, double *state, const uint8_t *in, uint8_t *out,
                     const uint32_t *s_c, uint64_t T)
{
    mt_job J = {H, W, C, n, r, pm, state, in, out, s_c, T, NULL, NULL};
    const uint64_t F = (uint64_t)H * W * C;
    J.work = (uint8_t *)malloc(F);
    J.conf = (uint8_t *)malloc(F);
    pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * n);
    mt_arg *args = (mt_arg *)malloc(sizeof(mt_arg) * n);
    int rc = -1;
    if (J.work && J.conf && th && args && pthread_barrier_init(&J.bar, NULL, n) == 0) {
        uint32_t started = 0;
        for (; started < n; started++) {
            args[started].job = &J;
            args[started].band = started;
            if (pthread_create(&th[started], NULL, mt_worker, &args[started]) != 0) break;
        }
        if (started == n) rc = 0;
        else abort();  /* a partial team would wait at the barrier for ever */
        for (uint32_t k = 0; k < started; k++) pthread_join(th[k], NULL);
        pthread_barrier_destroy(&J.bar);
    }
    free(J.work);
    free(J.conf);
    free(th);
    free(args);
    return rc;
}
