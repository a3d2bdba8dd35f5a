/*
 * oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, single-threaded CPU oracle of the real-time chaotic video
 * cipher of Jiang, Yuan, Li and Lu, "Real-time chaotic video encryption
 * based on multithreaded parallel confusion and diffusion" (arXiv 2302.07411).
 * It exists to check the GPU library bit for bit.  Only the test suite, the
 * smoke check and the CPU-baseline leg of the benchmark may load it; the GPU
 * library neither links nor calls it, and the two share no source.
 *
 * Every function follows the paper step by step, in its order and notation:
 *   - Sec. 3, Eq. (5): the piecewise linear chaotic map (PLCM);
 *   - Sec. 3, PLCM byte extraction (two PLCMs, 6 mantissa bytes of every
 *     iterate, the two byte sets XORed);
 *   - Sec. 3, Eq. (6): the 2D logistic-adjusted-sine map (2DLASM) and its
 *     byte extraction (two maps, 6 bytes of every x and every y iterate,
 *     XORed between the maps);
 *   - Sec. 2, Eq. (1) and Algorithm 2: confusion (discretised Chirikov map);
 *   - Sec. 2, Eq. (2): inverse confusion;
 *   - Sec. 2, Eq. (3) and Algorithm 2: diffusion with the seed taken from
 *     the next subframe;
 *   - Sec. 2, Eq. (4): inverse diffusion;
 *   - Sec. 2, Algorithms 1 and 2: r rounds of confusion then diffusion per
 *     frame, PRBG state carried across frames.
 * Where the paper is silent the oracle takes these readings (the same ones
 * the library documents in include/chaosvid.h):
 *   colour frames are interleaved HWC bytes; confusion moves whole pixels,
 *   diffusion chains over the band's bytes in memory order;
 *   band i covers rows [floor(i*H/n), floor((i+1)*H/n));
 *   non-square frames use alpha=(a+o) mod H, beta=(o+g(alpha)) mod W with
 *   g(alpha)=floor(s_c*sin((2*pi*alpha)/H)) evaluated in binary64;
 *   the diffusion seed is the last byte of the next band after confusion and
 *   before diffusion; "+" and "-" are mod 256;
 *   the 6 bytes are bytes 0..5 (least significant first) of the binary64
 *   bit pattern; the keystream of band i for one frame is the first r*S_i
 *   bytes of ceil(r*S_i/6) steps, round j consuming bytes [j*S_i,(j+1)*S_i).
 *
 * For Eq. (6) the oracle reads the products left to right,
 * (((pi*mu)*(y+3))*x)*(1-x) with pi = M_PI, and takes the sine correctly
 * rounded (RN(sin(t))): the sine is evaluated in binary128 by libquadmath
 * and rounded once to binary64; a value so close to a rounding boundary
 * that binary128 cannot decide it is reported, never guessed.
 *
 * Build: gcc -std=c11 -O2 -ffp-contract=off -fno-fast-math (SSE2 binary64,
 * no FMA contraction) -lquadmath, so every binary64 operation below is a
 * single correctly rounded IEEE-754 operation.
 */
#include <math.h>
#include <quadmath.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* ---------------------------------------------------------------- PLCM --- */

/* Sec. 3, Eq. (5): F(x,p) = x/p on [0,p); (x-p)/(1/2-p) on [p,1/2];
 * F(1-x,p) on (1/2,1]. */
double oracle_plcm(double x, double p)
{
    if (x < p)
        return x / p;
    if (x <= 0.5)
        return (x - p) / (0.5 - p);
    return oracle_plcm(1.0 - x, p);
}

static uint64_t bits_of(double x)
{
    uint64_t u;
    memcpy(&u, &x, sizeof u);
    return u;
}

/* Sec. 3, PLCM byte generator: iterate both PLCMs once per step (x_1, x_2,
 * ... -- the initial value itself is not emitted), take 6 bytes of each
 * iterate's mantissa field, XOR the byte of map 1 with the byte of map 2.
 * Writes exactly nbytes; the unused bytes of the last step are dropped.
 * *x1 and *x2 are advanced by ceil(nbytes/6) steps. */
void oracle_plcm_bytes(double *x1, double p1, double *x2, double p2,
                       uint64_t nbytes, uint8_t *out)
{
    uint64_t made = 0;
    while (made < nbytes) {
        *x1 = oracle_plcm(*x1, p1);
        *x2 = oracle_plcm(*x2, p2);
        uint64_t u = bits_of(*x1), v = bits_of(*x2);
        for (int k = 0; k < 6 && made < nbytes; k++)
            out[made++] = (uint8_t)(((u >> (8 * k)) & 0xFF) ^ ((v >> (8 * k)) & 0xFF));
    }
}

/* -------------------------------------------------------------- 2DLASM --- */

/* RN(sin(t)): sinq is accurate to about one binary128 ulp (2^-112 relative),
 * so rounding its value to binary64 gives the correctly rounded sine unless
 * it lies within 2^-100 of a binary64 midpoint; then 1 is returned and the
 * result must not be trusted.  (The margin is a parameter of the first
 * function only so that the test suite can exercise the check.) */
int oracle_cr_sin_margin(double t, double *out, int log2_margin)
{
    __float128 s = sinq((__float128)t);
    double d = (double)s;
    *out = d;
    if (s == 0)
        return 0;
    __float128 up = (__float128)nextafter(d, INFINITY);
    __float128 dn = (__float128)nextafter(d, -INFINITY);
    __float128 m_up = ((__float128)d + up) / 2, m_dn = ((__float128)d + dn) / 2;
    __float128 tol = fabsq(s) * ldexpq(1.0Q, log2_margin);
    return (fabsq(s - m_up) <= tol || fabsq(s - m_dn) <= tol) ? 1 : 0;
}

int oracle_cr_sin(double t, double *out)
{
    return oracle_cr_sin_margin(t, out, -100);
}

/* oracle_cr_sin over an array; returns the number of undecided values. */
uint64_t oracle_cr_sin_array(const double *t, double *out, uint64_t n)
{
    uint64_t bad = 0;
    for (uint64_t i = 0; i < n; i++)
        bad += (uint64_t)oracle_cr_sin(t[i], &out[i]);
    return bad;
}

/* Sec. 3, Eq. (6): x' = sin(pi*mu*(y+3)*x*(1-x)), then
 * y' = sin(pi*mu*(x'+3)*y*(1-y)) -- the new x enters the y update.
 * Returns 1 (state unchanged) if a sine could not be rounded with certainty. */
int oracle_lasm(double *x, double *y, double mu)
{
    double nx, ny;
    double ax = (((M_PI * mu) * (*y + 3.0)) * *x) * (1.0 - *x);
    if (oracle_cr_sin(ax, &nx))
        return 1;
    double ay = (((M_PI * mu) * (nx + 3.0)) * *y) * (1.0 - *y);
    if (oracle_cr_sin(ay, &ny))
        return 1;
    *x = nx;
    *y = ny;
    return 0;
}

/* Sec. 3, 2DLASM byte generator: per step both maps advance once; the
 * iterates are taken in the order x_1, y_1, x_2, y_2, ..., 6 bytes of each
 * (bytes 0..5 of the binary64 pattern), the bytes of map 1 XORed with those
 * of map 2: 12 bytes per step.  Writes exactly nbytes (the rest of the last
 * step is dropped); advances both maps by ceil(nbytes/12) steps.  Returns 1
 * if a sine could not be rounded with certainty. */
int oracle_lasm_bytes(double *x1, double *y1, double mu1, double *x2, double *y2,
                      double mu2, uint64_t nbytes, uint8_t *out)
{
    uint64_t k = 0;
    while (k < nbytes) {
        if (oracle_lasm(x1, y1, mu1) || oracle_lasm(x2, y2, mu2))
            return 1;
        uint64_t bx = bits_of(*x1) ^ bits_of(*x2);
        uint64_t by = bits_of(*y1) ^ bits_of(*y2);
        for (int b = 0; b < 6 && k < nbytes; b++)
            out[k++] = (uint8_t)(bx >> (8 * b));
        for (int b = 0; b < 6 && k < nbytes; b++)
            out[k++] = (uint8_t)(by >> (8 * b));
    }
    return 0;
}

/* ------------------------------------------------------ key schedule --- */

/* Algorithm 1: the main thread's PRBG_m, initialised with K, gives P_m and
 * then one s_c per frame.  The conversion is not given by the paper; this is
 * reading 1 (see the library's header): a draw is one step of the master
 * (PLCM master: both maps, (u, v) = (x_1, x_2); 2DLASM master: one map,
 * (u, v) = (x, y)); parameters come from draws with u and v in (0,1), band
 * after band -- PLCM (x0, p) = (u, v/2) per map; 2DLASM (x0, y0) = (u, v)
 * then mu = 0.44 + 0.49 u per map -- and after P_m every draw gives one
 * seed s_c = 1 + ((bits(u) XOR bits(v)) mod 2^16).
 * is_lasm = 0: K = {x0_1, p_1, x0_2, p_2}; 1: K = {x0, y0, mu}.
 * Returns 0, 1 (a sine undecided) or 2 (1000 unusable draws in a row). */
static int master_draw(int is_lasm, double *s, double *u, double *v)
{
    if (!is_lasm) {
        s[0] = oracle_plcm(s[0], s[1]);
        s[2] = oracle_plcm(s[2], s[3]);
        *u = s[0];
        *v = s[2];
        return 0;
    }
    if (oracle_lasm(&s[0], &s[1], s[2]))
        return 1;
    *u = s[0];
    *v = s[1];
    return 0;
}

static int master_usable(int is_lasm, double *s, double *u, double *v)
{
    for (int tries = 0; tries < 1000; tries++) {
        if (master_draw(is_lasm, s, u, v))
            return 1;
        if (*u > 0.0 && *u < 1.0 && *v > 0.0 && *v < 1.0)
            return 0;
    }
    return 2;
}

int oracle_key_schedule(int is_lasm, const double *K, uint32_t n, double *pm,
                        uint64_t first_frame, uint32_t *s_c, uint64_t T)
{
    double s[4] = {K[0], K[1], K[2], is_lasm ? 0.0 : K[3]};
    double u, v;
    int rc;
    for (uint32_t i = 0; i < n; i++) {
        for (int m = 0; m < 2; m++) {
            if ((rc = master_usable(is_lasm, s, &u, &v)))
                return rc;
            if (!is_lasm) {
                pm[4 * i + 2 * m] = u;
                pm[4 * i + 2 * m + 1] = v / 2.0;
            } else {
                pm[6 * i + 3 * m] = u;
                pm[6 * i + 3 * m + 1] = v;
                if ((rc = master_usable(is_lasm, s, &u, &v)))
                    return rc;
                pm[6 * i + 3 * m + 2] = 0.44 + 0.49 * u;
            }
        }
    }
    for (uint64_t t = 0; t < first_frame + T; t++) {
        if (master_draw(is_lasm, s, &u, &v))
            return 1;
        if (t >= first_frame)
            s_c[t - first_frame] = 1u + (uint32_t)((bits_of(u) ^ bits_of(v)) & 0xFFFFu);
    }
    return 0;
}

/* ------------------------------------------------------------ geometry --- */

/* Algorithm 2's band bounds (rows i*w/n up to (i+1)*w/n), generalised so
 * that every row is covered when n does not divide H. */
uint32_t oracle_band_lo(uint32_t H, uint32_t n, uint32_t i)
{
    return (uint32_t)(((uint64_t)i * H) / n);
}

static int64_t mod_nonneg(int64_t x, int64_t m)
{
    int64_t r = x % m;
    return r < 0 ? r + m : r;
}

/* Eq. (1): the shift s_c*sin(2*pi*alpha/w) of row alpha, floored to an
 * integer, in binary64 with the product and quotient taken left to right. */
void oracle_gtable(uint32_t H, uint32_t s_c, int64_t *g)
{
    for (uint32_t alpha = 0; alpha < H; alpha++) {
        double angle = ((2.0 * M_PI) * (double)alpha) / (double)H;
        g[alpha] = (int64_t)floor((double)s_c * sin(angle));
    }
}

/* ----------------------------------------------------------- confusion --- */

/* Eq. (1) for the source pixels of rows [a_lo, a_hi): every pixel (a,o) is
 * written to (alpha,beta) = ((a+o) mod H, (o+g[alpha]) mod W); the C bytes
 * of a pixel move together.  (Algorithm 2 has each subframe's thread move the
 * pixels of its own rows.) */
void oracle_confuse_rows(const uint8_t *in, uint8_t *out, uint32_t H, uint32_t W,
                         uint32_t C, const int64_t *g, uint32_t a_lo, uint32_t a_hi)
{
    for (uint32_t a = a_lo; a < a_hi; a++)
        for (uint32_t o = 0; o < W; o++) {
            int64_t alpha = mod_nonneg((int64_t)a + o, H);
            int64_t beta = mod_nonneg((int64_t)o + g[alpha], W);
            memcpy(out + ((uint64_t)alpha * W + beta) * C,
                   in + ((uint64_t)a * W + o) * C, C);
        }
}

/* Eq. (1) for the whole frame. */
void oracle_confuse(const uint8_t *in, uint8_t *out, uint32_t H, uint32_t W,
                    uint32_t C, const int64_t *g)
{
    oracle_confuse_rows(in, out, H, W, C, g, 0, H);
}

/* Eq. (2): pixel (alpha,beta) goes back to o=(beta-g[alpha]) mod W and
 * a=(alpha-o) mod H (for H=W this is a=(alpha-beta+g[alpha]) mod w). */
void oracle_unconfuse(const uint8_t *in, uint8_t *out, uint32_t H, uint32_t W,
                      uint32_t C, const int64_t *g)
{
    for (uint32_t alpha = 0; alpha < H; alpha++)
        for (uint32_t beta = 0; beta < W; beta++) {
            int64_t o = mod_nonneg((int64_t)beta - g[alpha], W);
            int64_t a = mod_nonneg((int64_t)alpha - o, H);
            memcpy(out + ((uint64_t)a * W + o) * C,
                   in + ((uint64_t)alpha * W + beta) * C, C);
        }
}

/* ----------------------------------------------------------- diffusion --- */

/* Keystream layout of one frame used by the oracle: the r*S_i bytes of band
 * i are stored from byte r*lo_i*W*C on (bands in order). */

/* Eq. (3) for band i of the frame, round j: its first byte is chained to
 * s_d, the last byte of band (i+1) mod n of the confused frame (before
 * diffusion); every other byte to the previous cipher byte. */
void oracle_diffuse_band(const uint8_t *Y, uint8_t *Z, uint32_t H, uint32_t W,
                         uint32_t C, uint32_t n, uint32_t r, uint32_t j,
                         const uint8_t *ks, uint32_t i)
{
    uint64_t row = (uint64_t)W * C;
    uint64_t lo = oracle_band_lo(H, n, i) * row;
    uint64_t hi = oracle_band_lo(H, n, i + 1) * row;
    uint64_t S = hi - lo;
    uint64_t next_hi = oracle_band_lo(H, n, (i + 1) % n + 1) * row;
    const uint8_t *b = ks + (uint64_t)r * lo + (uint64_t)j * S;
    uint8_t prev = Y[next_hi - 1]; /* s_d */
    for (uint64_t k = 0; k < S; k++) {
        uint8_t sum = (uint8_t)(Y[lo + k] + b[k]);
        Z[lo + k] = (uint8_t)(b[k] ^ sum ^ prev);
        prev = Z[lo + k];
    }
}

/* Eq. (3) for every band of the frame, round j. */
void oracle_diffuse(const uint8_t *Y, uint8_t *Z, uint32_t H, uint32_t W,
                    uint32_t C, uint32_t n, uint32_t r, uint32_t j,
                    const uint8_t *ks)
{
    for (uint32_t i = 0; i < n; i++)
        oracle_diffuse_band(Y, Z, H, W, C, n, r, j, ks, i);
}

/* Eq. (4): P = (b xor C xor C_prev) - b.  The seed of band i is recovered
 * first: it is the pre-diffusion last byte of band i'=(i+1) mod n, i.e.
 * Eq. (4) applied to that band's last byte (its predecessor lies in the same
 * band because every band holds at least 2 bytes). */
void oracle_undiffuse(const uint8_t *Z, uint8_t *Y, uint32_t H, uint32_t W,
                      uint32_t C, uint32_t n, uint32_t r, uint32_t j,
                      const uint8_t *ks)
{
    uint64_t row = (uint64_t)W * C;
    for (uint32_t i = 0; i < n; i++) {
        uint64_t lo = oracle_band_lo(H, n, i) * row;
        uint64_t hi = oracle_band_lo(H, n, i + 1) * row;
        uint64_t S = hi - lo;
        uint32_t ip = (i + 1) % n;
        uint64_t lo_p = oracle_band_lo(H, n, ip) * row;
        uint64_t hi_p = oracle_band_lo(H, n, ip + 1) * row;
        uint64_t S_p = hi_p - lo_p;
        uint8_t bp = ks[(uint64_t)r * lo_p + (uint64_t)j * S_p + S_p - 1];
        uint8_t s_d = (uint8_t)((bp ^ Z[hi_p - 1] ^ Z[hi_p - 2]) - bp);
        const uint8_t *b = ks + (uint64_t)r * lo + (uint64_t)j * S;
        for (uint64_t k = 0; k < S; k++) {
            uint8_t prev = k ? Z[lo + k - 1] : s_d;
            Y[lo + k] = (uint8_t)((b[k] ^ Z[lo + k] ^ prev) - b[k]);
        }
    }
}

/* ------------------------------------------------------ whole frames --- */

/* Algorithm 2, first two steps of the frame loop: the keystream of every
 * band for T frames (r*F bytes per frame in the layout above).  x1, x2 hold
 * the n chain states and are advanced. */
void oracle_plcm_keystream(uint32_t H, uint32_t W, uint32_t C, uint32_t n,
                           uint32_t r, double *x1, const double *p1,
                           double *x2, const double *p2, uint64_t T,
                           uint8_t *ks)
{
    uint64_t row = (uint64_t)W * C, F = (uint64_t)H * row;
    for (uint64_t t = 0; t < T; t++)
        for (uint32_t i = 0; i < n; i++) {
            uint64_t lo = oracle_band_lo(H, n, i) * row;
            uint64_t S = oracle_band_lo(H, n, i + 1) * row - lo;
            oracle_plcm_bytes(&x1[i], p1[i], &x2[i], p2[i], (uint64_t)r * S,
                              ks + t * (uint64_t)r * F + (uint64_t)r * lo);
        }
}

/* The 2DLASM keystream of T frames in the layout of oracle_plcm_keystream;
 * each band's records (x1,y1,mu1,x2,y2,mu2) advance.  Returns 1 if a sine
 * could not be rounded with certainty. */
int oracle_lasm_keystream(uint32_t H, uint32_t W, uint32_t C, uint32_t n, uint32_t r,
                          double *x1, double *y1, const double *mu1, double *x2,
                          double *y2, const double *mu2, uint64_t T, uint8_t *ks)
{
    uint64_t row = (uint64_t)W * C, F = (uint64_t)H * row;
    for (uint64_t t = 0; t < T; t++)
        for (uint32_t i = 0; i < n; i++) {
            uint64_t lo = oracle_band_lo(H, n, i) * row;
            uint64_t S = oracle_band_lo(H, n, i + 1) * row - lo;
            if (oracle_lasm_bytes(&x1[i], &y1[i], mu1[i], &x2[i], &y2[i], mu2[i],
                                  (uint64_t)r * S, ks + t * (uint64_t)r * F + (uint64_t)r * lo))
                return 1;
        }
    return 0;
}

/* The rounds of Algorithm 2 for T frames whose keystream is given (r*F
 * bytes per frame): encryption confuses (Eq. 1) then diffuses (Eq. 3) r
 * times; decryption undoes diffusion (Eq. 4) then confusion (Eq. 2) in
 * reverse round order. */
int oracle_rounds(uint32_t H, uint32_t W, uint32_t C, uint32_t n, uint32_t r, int decrypt,
                  const uint8_t *ks, const uint8_t *in, uint8_t *out, const uint32_t *s_c,
                  uint64_t T)
{
    uint64_t F = (uint64_t)H * W * C;
    uint8_t *A = malloc(F), *Y = malloc(F);
    int64_t *g = malloc(sizeof(int64_t) * H);
    if (!A || !Y || !g) {
        free(A); free(Y); free(g);
        return -1;
    }
    for (uint64_t t = 0; t < T; t++) {
        const uint8_t *k = ks + t * (uint64_t)r * F;
        oracle_gtable(H, s_c[t], g);
        memcpy(A, in + t * F, F);
        if (!decrypt) {
            for (uint32_t j = 0; j < r; j++) {
                oracle_confuse(A, Y, H, W, C, g);
                oracle_diffuse(Y, A, H, W, C, n, r, j, k);
            }
        } else {
            for (uint32_t jj = r; jj-- > 0;) {
                oracle_undiffuse(A, Y, H, W, C, n, r, jj, k);
                oracle_unconfuse(Y, A, H, W, C, g);
            }
        }
        memcpy(out + t * F, A, F);
    }
    free(A); free(Y); free(g);
    return 0;
}

/* Algorithms 1 and 2: for every frame, generate the keystream, then r times
 * confuse the whole frame (Eq. 1) and diffuse every band (Eq. 3).  The
 * confusion seed s_c[t] is the same for all rounds of frame t. */
int oracle_encrypt(uint32_t H, uint32_t W, uint32_t C, uint32_t n, uint32_t r,
                   double *x1, const double *p1, double *x2, const double *p2,
                   const uint8_t *in, uint8_t *out, const uint32_t *s_c,
                   uint64_t T)
{
    uint64_t F = (uint64_t)H * W * C;
    uint8_t *ks = malloc((uint64_t)r * F), *A = malloc(F), *Y = malloc(F);
    int64_t *g = malloc(sizeof(int64_t) * H);
    if (!ks || !A || !Y || !g) {
        free(ks); free(A); free(Y); free(g);
        return -1;
    }
    for (uint64_t t = 0; t < T; t++) {
        oracle_plcm_keystream(H, W, C, n, r, x1, p1, x2, p2, 1, ks);
        oracle_gtable(H, s_c[t], g);
        memcpy(A, in + t * F, F);
        for (uint32_t j = 0; j < r; j++) {
            oracle_confuse(A, Y, H, W, C, g);
            oracle_diffuse(Y, A, H, W, C, n, r, j, ks);
        }
        memcpy(out + t * F, A, F);
    }
    free(ks); free(A); free(Y); free(g);
    return 0;
}

/* Decryption: the same keystream, then the rounds in reverse order, each
 * undoing diffusion (Eq. 4) and then confusion (Eq. 2). */
int oracle_decrypt(uint32_t H, uint32_t W, uint32_t C, uint32_t n, uint32_t r,
                   double *x1, const double *p1, double *x2, const double *p2,
                   const uint8_t *in, uint8_t *out, const uint32_t *s_c,
                   uint64_t T)
{
    uint64_t F = (uint64_t)H * W * C;
    uint8_t *ks = malloc((uint64_t)r * F), *A = malloc(F), *Y = malloc(F);
    int64_t *g = malloc(sizeof(int64_t) * H);
    if (!ks || !A || !Y || !g) {
        free(ks); free(A); free(Y); free(g);
        return -1;
    }
    for (uint64_t t = 0; t < T; t++) {
        oracle_plcm_keystream(H, W, C, n, r, x1, p1, x2, p2, 1, ks);
        oracle_gtable(H, s_c[t], g);
        memcpy(A, in + t * F, F);
        for (uint32_t jj = r; jj-- > 0;) {
            oracle_undiffuse(A, Y, H, W, C, n, r, jj, ks);
            oracle_unconfuse(Y, A, H, W, C, g);
        }
        memcpy(out + t * F, A, F);
    }
    free(ks); free(A); free(Y); free(g);
    return 0;
}
