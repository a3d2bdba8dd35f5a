/*
 * chaosvid.h -- C ABI of libchaosvid, a GPU (AMD Instinct MI355X, gfx950)
 * implementation of the real-time chaotic video cipher of Jiang, Yuan, Li
 * and Lu, "Real-time chaotic video encryption based on multithreaded
 * parallel confusion and diffusion" (arXiv 2302.07411).
 *
 * The cipher (Sec. 2, Algorithms 1-2): every frame is split into n
 * horizontal subframes (bands); each band owns a chaotic byte generator
 * whose state runs on from frame to frame.  A frame is encrypted by r rounds
 * of confusion (Eq. 1: a whole-frame pixel permutation, the discretised
 * Chirikov map with the frame's confusion seed s_c) followed by diffusion
 * (Eq. 3: every band chains its bytes with the generator's bytes, seeded by
 * the last byte of the next band).  Decryption applies Eq. (4) and Eq. (2)
 * in reverse order.  The byte generator is the PLCM pair of Sec. 3 (Eq. 5).
 *
 * Readings where the paper is silent (fixed here, and what the CPU oracle of
 * the test suite implements):
 *  - frames are 8-bit, HWC interleaved (OpenCV order); confusion moves whole
 *    pixels; diffusion chains over a band's bytes in memory order;
 *  - band i covers rows [floor(i*H/n), floor((i+1)*H/n));
 *  - for H != W: alpha=(a+o) mod H, beta=(o+g(alpha)) mod W;
 *  - g(alpha) = floor(s_c*sin((2*pi*alpha)/H)) in binary64, evaluated left
 *    to right (on the host, with the C library's sin);
 *  - the diffusion seed of band i is the last byte of band (i+1) mod n after
 *    confusion and before diffusion; + and - are mod 256;
 *  - a PLCM step emits bytes 0..5 (least significant first) of each map's
 *    binary64 iterate, XORed between the two maps; the first iterate x_1 is
 *    the first one used; per frame band i takes the first r*S_i bytes of
 *    ceil(r*S_i/6) steps (S_i = bytes of band i), round j using bytes
 *    [j*S_i, (j+1)*S_i).
 *
 * Conventions.  All functions return cv_status; no C++ exception crosses the
 * ABI.  On error the key state is unchanged and cv_last_error() (thread
 * local) describes the failure.  Frame and keystream buffers are DEVICE
 * pointers owned by the caller; `stream` is a hipStream_t (NULL = the null
 * stream).  Calls that take a stream are asynchronous and stream-ordered.
 * A key is not thread-safe.  Errors reported by the HIP runtime surface as
 * CV_E_HIP, asynchronous ones on a later call.
 */
#ifndef CHAOSVID_H
#define CHAOSVID_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CV_SPEC_VERSION 1

typedef enum {
  CV_OK = 0,
  CV_E_INVAL = 1, /* invalid argument (see each function) */
  CV_E_NOMEM = 2, /* device or pinned host allocation failed */
  CV_E_HIP = 3,   /* the HIP runtime reported an error */
  CV_E_AGAIN = 4, /* no capacity right now, retry later */
  CV_E_STATE = 5  /* the object is in the wrong state for the call */
} cv_status;

typedef enum {
  CV_MAP_PLCM = 0 /* two piecewise linear chaotic maps per band (Sec. 3, Eq. 5) */
} cv_map;

/* Round implementation used by cv_encrypt_frames / cv_decrypt_frames.
 * Both give identical bytes. */
typedef enum {
  CV_PATH_PLAIN = 0, /* one kernel launch per round over the batch of frames */
  CV_PATH_FUSED = 1  /* all r rounds in one persistent launch per batch: groups of n
                        workgroups (one per subframe) exchange bands through on-chip
                        cached scratch with a group barrier per round (Algorithm 1's
                        round loop on the device).  Needs the pixel-word conditions
                        (C in {3,4}, W % 16 == 0, 16-byte aligned buffers); other
                        geometries run the plain path. */
} cv_path;

/* Frame geometry: height H, width W, channels C (bytes per pixel), number of
 * subframes n (Algorithm 1's assistant threads) and rounds r (Sec. 6 uses 5). */
typedef struct {
  uint32_t height, width, channels, n_sub, rounds;
} cv_geom;

typedef struct cv_key cv_key;

/* Launch shape of a key's kernels.  Any choice gives identical bytes; it
 * only moves work between batches, workgroups and LDS tiles. */
typedef struct {
  uint32_t batch_frames;   /* frames per internal batch (keystream + scratch workspace) */
  uint32_t threads;        /* threads per round workgroup: 64..1024, multiple of 64 */
  uint32_t tile_rows_enc;  /* frame rows staged in LDS per step of an encryption round */
  uint32_t tile_rows_dec;  /* frame rows staged in LDS per step of a decryption round */
  uint32_t prbg_variant;   /* keystream generator, all giving the same bytes:
                              0 auto (fastest valid), 1 IEEE division instruction sequence,
                              2 reciprocal + two FMA corrections (provably correctly rounded
                                for keys with p >= 2^-64 and states 0 or >= 2^-800),
                              3 as 2 with one lane per piece of the map.
                              2 and 3 fall back to 1 for keys outside that domain. */
  uint32_t round_variant;  /* round kernels, all giving the same bytes: 0 auto, 1 byte
                              kernels (any geometry), 2 pixel-word kernels (C in {3,4},
                              W a multiple of 16, 16-byte aligned buffers; otherwise 1) */
  uint32_t tile_rows_pw;   /* frame rows per LDS tile of the pixel-word kernels */
  uint32_t fused_groups;   /* CV_PATH_FUSED: frame groups in flight (multiple of 8); 0 = as
                              many as can be resident (reading back gives the value used) */
} cv_launch;

/* Version of the cipher readings above (CV_SPEC_VERSION). */
int cv_spec_version(void);

/* Message of the last failed call on this thread ("" if none). */
const char *cv_last_error(void);

/* Set up the per-band generators of one video stream (Algorithm 2,
 * "Initialize PRBG_a^i with p_m^i"; Sec. 3, Eq. 5).
 *  geom      frame geometry; requires H,W,C,n,r >= 1, n <= H, every band at
 *            least 2 bytes, H*W*C < 2^32 per row block limits of uint32.
 *  map       CV_MAP_PLCM.
 *  p_m       host array of n records {x0_1, p_1, x0_2, p_2} (map 1, map 2);
 *            x0 in (0,1), p in (0,1/2), all finite.
 *  n_doubles 4*n.
 *  device    HIP device ordinal the key lives on.
 *  out       receives the key (owned by the caller, release with cv_key_free).
 * Errors: CV_E_INVAL for any violated requirement, CV_E_NOMEM, CV_E_HIP. */
cv_status cv_keysetup(const cv_geom *geom, cv_map map, const double *p_m, size_t n_doubles,
                      int device, cv_key **out);

/* Release a key and its device memory (synchronises the device first).
 * NULL is ignored. */
void cv_key_free(cv_key *key);

/* Current generator state (Algorithm 2: the PRBG state persists from frame
 * to frame) for checkpointing: x holds n records {x_1, x_2} (2*n doubles),
 * *frame_index the number of frames processed so far.  Synchronises the
 * key's device.  CV_E_INVAL if n_doubles != 2*n or a pointer is NULL. */
cv_status cv_key_get_state(const cv_key *key, double *x, size_t n_doubles, uint64_t *frame_index);

/* Restore a state obtained from cv_key_get_state (same geometry and p_m).
 * Synchronises the key's device.  CV_E_INVAL as above or if any x is
 * outside [0,1]. */
cv_status cv_key_set_state(cv_key *key, const double *x, size_t n_doubles, uint64_t frame_index);

/* Choose the round implementation (CV_PATH_*).  CV_E_INVAL if unknown. */
cv_status cv_key_set_path(cv_key *key, int path);

/* Read the key's launch shape (chosen at cv_keysetup from the geometry and
 * the device's LDS size). */
cv_status cv_key_get_launch(const cv_key *key, cv_launch *launch);

/* Set the launch shape.  CV_E_INVAL if batch_frames = 0, threads is not a
 * multiple of 64 in 64..1024, a tile is 0 rows, larger than threads, or
 * needs more LDS than one workgroup may have.  Tile rows beyond a band's
 * height (encryption) or the frame height (decryption) are clamped. */
cv_status cv_key_set_launch(cv_key *key, const cv_launch *launch);

/* Per-kernel timing of a key's launches, accumulated while profiling is on:
 * HIP events are recorded on the launch stream around every kernel. */
typedef struct {
  double prbg_ms;        /* keystream generator launches */
  uint64_t prbg_launches;
  uint64_t prbg_steps;   /* chain steps (two PLCM iterates each) generated */
  double round_ms;       /* confusion+diffusion round launches (both directions) */
  uint64_t round_launches;
  uint64_t round_frames; /* frame-rounds processed */
} cv_profile;

/* Turn event profiling on (1) or off (0); turning it on clears the totals. */
cv_status cv_key_set_profiling(cv_key *key, int on);

/* Totals since profiling was turned on (synchronises the recorded events).
 * CV_E_STATE if profiling is off. */
cv_status cv_key_get_profile(cv_key *key, cv_profile *prof);

/* Encrypt n_frames consecutive frames of the stream (Algorithm 1 and 2):
 * for every frame, generate its keystream, then r rounds of confusion
 * (Eq. 1) and diffusion (Eq. 3).
 *  in, out   device buffers of n_frames*H*W*C bytes, HWC frames back to
 *            back; must not overlap.
 *  s_c       host array of n_frames confusion seeds (Algorithm 1, "generate
 *            a confusion seed s_c"), each >= 1.
 *  stream    hipStream_t the work is ordered on.
 * Advances the key by n_frames frames.  n_frames = 0 is a no-op.
 * Errors: CV_E_INVAL (NULL, overlap, s_c = 0), CV_E_NOMEM, CV_E_HIP. */
cv_status cv_encrypt_frames(cv_key *key, const uint8_t *in, uint8_t *out, const uint32_t *s_c,
                            size_t n_frames, void *stream);

/* Decrypt n_frames frames encrypted with a key built from the same p_m, fed
 * in the same order with the same s_c (Eq. 4 then Eq. 2, rounds reversed).
 * Same arguments and errors as cv_encrypt_frames. */
cv_status cv_decrypt_frames(cv_key *key, const uint8_t *in, uint8_t *out, const uint32_t *s_c,
                            size_t n_frames, void *stream);

/* Write the keystream of the next n_frames frames into ks (device, n_frames
 * * r*H*W*C bytes; per frame band i's r*S_i bytes start at byte
 * r*floor(i*H/n)*W*C) and advance the key (Algorithm 2, "Iterate PRBG_a^i,
 * generate enough iteration results; convert them into byte sequence B_i").
 * Errors: CV_E_INVAL (NULL), CV_E_HIP. */
cv_status cv_keystream_frames(cv_key *key, uint8_t *ks, size_t n_frames, void *stream);

/* The r rounds alone with a caller-supplied keystream in the layout of
 * cv_keystream_frames (Algorithm 2's round loop): decrypt = 0 encrypts
 * (Eq. 1 + Eq. 3, j = 0..r-1), decrypt = 1 decrypts (Eq. 4 + Eq. 2, j =
 * r-1..0).  Uses the key's geometry and workspace but not its generator
 * state, which is left unchanged.  Same buffer rules and errors as
 * cv_encrypt_frames; ks must not overlap in/out. */
cv_status cv_apply_rounds(cv_key *key, int decrypt, const uint8_t *in, uint8_t *out,
                          const uint8_t *ks, const uint32_t *s_c, size_t n_frames, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* CHAOSVID_H */
