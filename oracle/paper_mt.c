/*
 * paper_mt.c -- CPU BASELINE, TEST INFRASTRUCTURE ONLY.
 *
 * The paper's multithreaded CPU design of the cipher (Sec. 2: one assistant
 * thread per subframe, two barriers per round; its speed is what Sec. 3
 * measures), used to time that design on the host of the GPU machine and
 * checked against the single-threaded oracle.  It is built from the
 * oracle's pinned steps -- the PLCM byte generator of Eq. (5), the band
 * bounds, the shift table of Eq. (1), and Eq. (1) and Eq. (3) restricted to
 * one subframe (oracle_confuse_rows, oracle_diffuse_band) -- and shares
 * nothing with the GPU library.
 *
 * Thread i owns subframe i and its generator pair.  Per frame it writes its
 * subframe's r*S_i keystream bytes into the frame's keystream (at the
 * oracle's offset for band i) and computes its own copy of the row shifts;
 * per round it moves the pixels of its rows into the shared confused frame
 * (Eq. 1), waits until every thread has, chains its subframe (Eq. 3, seeded
 * from the next subframe of the confused frame), and waits again before the
 * next round reads the result.  The readings are the oracle's.
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
void oracle_confuse_rows(const uint8_t *in, uint8_t *out, uint32_t H, uint32_t W,
                         uint32_t C, const int64_t *g, uint32_t a_lo, uint32_t a_hi);
void oracle_diffuse_band(const uint8_t *Y, uint8_t *Z, uint32_t H, uint32_t W,
                         uint32_t C, uint32_t n, uint32_t r, uint32_t j,
                         const uint8_t *ks, uint32_t i);

typedef struct {
    uint32_t H, W, C, n, r;
    const double *pm;     /* n records (x0_1, p_1, x0_2, p_2); p used */
    double *state;        /* n pairs (x_1, x_2), advanced */
    const uint8_t *in;
    uint8_t *out;
    const uint32_t *s_c;
    uint64_t T;
    uint8_t *work;        /* the frame between rounds */
    uint8_t *conf;        /* the confused frame of the current round */
    uint8_t *ks;          /* the current frame's keystream, r*F bytes */
    pthread_barrier_t bar;
} mt_job;

typedef struct {
    mt_job *job;
    uint32_t band;
} mt_arg;

static void *mt_worker(void *p)
{
    const mt_arg *arg = (const mt_arg *)p;
    mt_job *J = arg->job;
    const uint32_t i = arg->band, H = J->H, W = J->W, C = J->C, n = J->n, r = J->r;
    const uint64_t row = (uint64_t)W * C, F = (uint64_t)H * row;
    const uint32_t lo = oracle_band_lo(H, n, i), hi = oracle_band_lo(H, n, i + 1);
    const uint64_t S = (uint64_t)(hi - lo) * row;
    int64_t *g = (int64_t *)malloc(sizeof(int64_t) * H);
    if (!g) abort();  /* a small allocation; a thread that cannot proceed would stall the team */
    for (uint64_t t = 0; t < J->T; t++) {
        /* this subframe's bytes only: no other thread reads them */
        oracle_plcm_bytes(&J->state[2 * i], J->pm[4 * i + 1], &J->state[2 * i + 1],
                          J->pm[4 * i + 3], r * S, J->ks + (uint64_t)r * lo * row);
        oracle_gtable(H, J->s_c[t], g);
        for (uint32_t j = 0; j < r; j++) {
            const uint8_t *src = j == 0 ? J->in + t * F : J->work;
            uint8_t *dst = j + 1 == r ? J->out + t * F : J->work;
            oracle_confuse_rows(src, J->conf, H, W, C, g, lo, hi);
            pthread_barrier_wait(&J->bar);  /* the confused frame is complete */
            oracle_diffuse_band(J->conf, dst, H, W, C, n, r, j, J->ks, i);
            pthread_barrier_wait(&J->bar);  /* the round's output is complete */
        }
    }
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
    mt_job J = {H, W, C, n, r, pm, state, in, out, s_c, T, NULL, NULL, NULL};
    const uint64_t F = (uint64_t)H * W * C;
    J.work = (uint8_t *)malloc(F);
    J.conf = (uint8_t *)malloc(F);
    J.ks = (uint8_t *)malloc(r * F);
    pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * n);
    mt_arg *args = (mt_arg *)malloc(sizeof(mt_arg) * n);
    int rc = -1;
    if (J.work && J.conf && J.ks && th && args && pthread_barrier_init(&J.bar, NULL, n) == 0) {
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
    free(J.ks);
    free(th);
    free(args);
    return rc;
}
