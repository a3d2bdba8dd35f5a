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
 *    [j*S_i, (j+1)*S_i);
 *  - a 2DLASM step computes x' = sin(((pi*mu)*(y+3))*x*(1-x)) and then
 *    y' = sin(((pi*mu)*(x'+3))*y*(1-y)) in binary64 from left to right
 *    (pi = M_PI) with the sine correctly rounded, and emits bytes 0..5 of
 *    x'(map 1) XOR x'(map 2), then bytes 0..5 of y'(map 1) XOR y'(map 2):
 *    12 bytes per step, ceil(r*S_i/12) steps per band and frame.
 *
 * Conventions.  All functions return cv_status; no C++ exception crosses the
 * ABI.  On an error found when a call is made (arguments, allocation, a
 * launch the runtime refuses) the key state is unchanged and cv_last_error()
 * (thread local) describes the failure.  Frame and keystream buffers are
 * DEVICE pointers owned by the caller; `stream` is a hipStream_t (NULL = the
 * null stream).  Calls that take a stream are asynchronous and
 * stream-ordered.  A key is not thread-safe.  Successive calls on one key
 * may take different streams: a call on another stream than the key's last
 * call waits for that call's work (the key's generator state and workspace
 * are shared).  A cv_batch_run tick likewise waits for its keys' earlier
 * calls; a call on a key after a tick that used it, on another stream than
 * the tick's, must be ordered by the caller (cv_batch_sync, or an event).
 * Work captured into a caller's own graph is ordered by the caller.
 *
 * Asynchronous device errors.  A fused launch whose group barrier times out
 * (or finds a group spread over XCDs) and a 2DLASM sine that cannot be
 * rounded with certainty set the key's device error word; the call that
 * enqueued that work has already returned CV_OK.  The error is reported, as
 * CV_E_HIP, by the first later call on the key that finds the word's
 * read-back complete (cv_key_sync, cv_key_get_state and cv_key_set_state
 * always wait for it); calls made before that may also return CV_OK.  From
 * the failing launch on, every output of the key is invalid, and after the
 * report the key is dead: every call that uses it fails with CV_E_STATE.
 * Free it and set up a new key (the generator state of a 2DLASM key that
 * failed is itself invalid).  A caller that must know that a batch of frames
 * is valid calls cv_key_sync after it.
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
  CV_MAP_PLCM = 0,  /* two piecewise linear chaotic maps per band (Sec. 3, Eq. 5) */
  CV_MAP_2DLASM = 1 /* two 2D logistic-adjusted-sine maps per band (Sec. 3, Eq. 6) */
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
                              0 auto (fastest valid: 4 where allowed, else 1),
                              1 IEEE division instruction sequence,
                              2 reciprocal + two FMA corrections (provably correctly rounded
                                for keys with p >= 2^-64 and states 0 or >= 2^-800),
                              3 as 2 with one lane per piece of the map,
                              4 two-operation quotient (multiply + FMA with a double-word
                                reciprocal) on the chain, every step recomputed from
                                checkpoints and checked against 2 by other wavefronts and
                                repaired from the first mismatch,
                              5 as 4 with a one-bit error planted in every 29th producer
                                step of every map and in every other one of those steps
                                of the verifiers' recomputation (testing both checks and
                                the repair; slower).
                              2..5 fall back to 1 for keys outside 2's domain. */
  uint32_t round_variant;  /* round kernels, all giving the same bytes: 0 auto (3 where it
                              applies), 1 byte kernels (any geometry), 2 pixel-word kernels
                              (C in {3,4}, W a multiple of 16, 16-byte aligned buffers;
                              otherwise 1), 3 as 2, with CV_PATH_FUSED encryption by whole
                              source-row runs and packed-byte diffusion, and decryption by
                              whole source-row runs: in one pass per subframe when every
                              subframe fits the LDS as one tile (4*(W+4) bytes per row plus
                              4*H), else tile by tile with the multi-stream kernel */
  uint32_t tile_rows_pw;   /* frame rows per LDS tile of the pixel-word kernels */
  uint32_t fused_groups;   /* CV_PATH_FUSED: frame groups in flight (multiple of 8); 0 = as
                              many as can be resident (reading back gives the value used) */
  uint32_t use_graph;      /* 1: cv_encrypt_frames / cv_decrypt_frames replay one HIP graph
                              per internal batch (shift-table copy, keystream launch, round
                              launches, error read-back), captured the first time a buffer
                              set (in, out, frame count, direction) is seen; up to 16 graphs
                              are kept, the least recently used dropped.  0: every kernel
                              launched on its own.  Ignored while profiling is on, and with
                              lookahead. */
  uint32_t lookahead;      /* 1 (PLCM and 2DLASM keys): after each internal
                              batch of T frames, generate the next T frames' keystream on a
                              private stream from a copy of the generator states made on the
                              call's stream (the keystream depends only on them, Algorithm 2),
                              so that a call arriving later finds it ready and costs only its
                              rounds.  The next batch takes it when it starts at the predicted
                              frame with the same T and the state was not set in between;
                              otherwise it is dropped.  The private stream never touches the
                              key's state.  Beside a call stream other than the null stream
                              it is a stream with a hardware queue of its own (a compute-unit
                              mask of every CU), so the call stream's later work never queues
                              behind a lookahead (such a stream is ordered with the legacy
                              null stream: null-stream work issued meanwhile waits for the
                              lookahead); beside the null stream it is a non-blocking stream.
                              Costs two keystream buffers of T frames.  0: off */
} cv_launch;

/* Version of the cipher readings above (CV_SPEC_VERSION). */
int cv_spec_version(void);

/* Message of the last failed call on this thread ("" if none). */
const char *cv_last_error(void);

/* Set up the per-band generators of one video stream (Algorithm 2: each
 * subframe's generator starts from its record of P_m; Sec. 3, Eq. 5).
 *  geom      frame geometry; requires H,W,C,n,r >= 1, n <= H, every band at
 *            least 2 bytes, H*W*C < 2^32 per row block limits of uint32.
 *  map       CV_MAP_PLCM or CV_MAP_2DLASM.
 *  p_m       host array of n records: PLCM {x0_1, p_1, x0_2, p_2} with x0 in
 *            (0,1), p in (0,1/2); 2DLASM {x0_1, y0_1, mu_1, x0_2, y0_2, mu_2}
 *            with x0, y0 in (0,1) and mu in [0.37,0.38], [0.4,0.42],
 *            [0.44,0.93] or {1} (Sec. 3, Eq. 6); all finite.
 *  n_doubles 4*n (PLCM) or 6*n (2DLASM).
 *  device    HIP device ordinal the key lives on.
 *  out       receives the key (owned by the caller, release with cv_key_free).
 * Errors: CV_E_INVAL for any violated requirement, CV_E_NOMEM, CV_E_HIP. */
cv_status cv_keysetup(const cv_geom *geom, cv_map map, const double *p_m, size_t n_doubles,
                      int device, cv_key **out);

/* The correctly rounded binary64 sine of the 2DLASM generator, RN(sin(t)),
 * exported so that it can be checked against an independent reference.
 * t, out: device arrays of n doubles, each t in [0, RN(pi)] (the range of
 * Eq. 6's arguments).  Three stages: a light evaluation (relative error
 * below 2^-69.2) with a rounding test, then the double-double fast path
 * (2^-100), then the 256-bit exact path.  force_exact = 1 skips the first
 * stage and evaluates every argument >= 2^-30 on the exact path.
 * *undecided (a device word the caller zeroes) is set to 1 if a value could
 * not be rounded with certainty.  Errors: CV_E_INVAL (NULL), CV_E_HIP. */
/* The first stage of cv_cr_sin on the host, for checking its error bound:
 * for each t (host arrays of n values, t in [0, RN(pi)]), hi + lo is the
 * stage's double-double approximation of sin(t) and decided[i] = 1 when its
 * rounding test accepts hi as RN(sin t) (otherwise the later stages decide).
 * No device is used.  Errors: CV_E_INVAL (NULL, t outside [0, RN(pi)]). */
cv_status cv_sin_stage1(const double *t, double *hi, double *lo, int *decided, size_t n);

cv_status cv_cr_sin(const double *t, double *out, size_t n, int force_exact, uint32_t *undecided,
                    void *stream);

/* Key schedule of the main thread (Algorithm 1): PRBG_m, initialised with the
 * key K, yields the parameters P_m of the n subframe generators and then one
 * confusion seed s_c per frame.  The paper leaves the conversion of iterates
 * into parameters open; reading CV_KEY_SCHEDULE_VERSION 1:
 *  - PLCM master: K = {x0_1, p_1, x0_2, p_2} (ranges as a PLCM record), two
 *    PLCMs (Eq. 5); a draw advances both and gives (u, v) = their iterates.
 *    2DLASM master: K = {x0, y0, mu} (the paper's three doubles), one 2DLASM
 *    (Eq. 6, correctly rounded sine); a draw is one step, (u, v) = (x, y).
 *  - P_m, band after band, from usable draws (u and v both in (0,1); other
 *    draws are skipped): PLCM records {x0_1, p_1, x0_2, p_2} take two draws,
 *    (x0, p) = (u, v/2) each; 2DLASM records {x0_1, y0_1, mu_1, x0_2, y0_2,
 *    mu_2} take two draws per map, (x0, y0) = (u, v), then
 *    mu = 0.44 + 0.49*u (inside the admissible [0.44, 0.93]).
 *  - Then one draw per frame, usable or not: s_c = 1 + ((bits(u) XOR
 *    bits(v)) mod 2^16), bits() the binary64 pattern.
 *  p_m       host array of 4*n_sub (PLCM) or 6*n_sub (2DLASM) doubles.
 *  s_c       host array of n_frames seeds for frames first_frame ...
 *            first_frame + n_frames - 1 (the earlier draws are generated and
 *            dropped), so a stream can be resumed at any frame.
 * Host computation; no device is used, and nothing is written on error
 * beyond the output arrays.  Errors: CV_E_INVAL (NULL, ranges, sizes, a
 * degenerate master orbit: 0 is a fixed point of both maps, so after 1000
 * consecutive unusable draws the key is rejected); CV_E_HIP if a 2DLASM sine
 * could not be rounded with certainty (the status the device generator
 * reports for the same event). */
#define CV_KEY_SCHEDULE_VERSION 1
cv_status cv_key_schedule(cv_map map, const double *K, size_t n_k, uint32_t n_sub, double *p_m,
                          size_t n_pm, uint64_t first_frame, uint32_t *s_c, size_t n_frames);

/* Release a key and its device memory (synchronises the device first).
 * NULL is ignored. */
void cv_key_free(cv_key *key);

/* Current generator state (Algorithm 2: the PRBG state persists from frame
 * to frame) for checkpointing: x holds n records, {x_1, x_2} for PLCM (2*n
 * doubles) or {x_1, y_1, x_2, y_2} for 2DLASM (4*n doubles), *frame_index
 * the number of frames processed so far.  Synchronises the key's device.
 * CV_E_INVAL if n_doubles is not that size or a pointer is NULL. */
cv_status cv_key_get_state(const cv_key *key, double *x, size_t n_doubles, uint64_t *frame_index);

/* Restore a state obtained from cv_key_get_state (same geometry and p_m).
 * Synchronises the key's device.  CV_E_INVAL as above or if any x is
 * outside [0,1]. */
cv_status cv_key_set_state(cv_key *key, const double *x, size_t n_doubles, uint64_t frame_index);

/* Wait for all work queued on the key's device and report the key's
 * asynchronous device errors (see the conventions above): CV_OK if every
 * frame the key has produced so far is valid, CV_E_HIP on the first report,
 * CV_E_STATE afterwards. */
cv_status cv_key_sync(cv_key *key);

/* Testing hook: polls of the fused path's group barrier before it gives up
 * and raises the key's device error (default 2^21, about two seconds).  With
 * 0 and n >= 2 subframes the first workgroup to reach a barrier gives up, so
 * every fused launch fails and every kernel still exits normally. */
cv_status cv_key_set_spin_limit(cv_key *key, uint32_t polls);

/* Choose the key's fused-path launch shape for batches of n_frames frames
 * in one direction: time the fused round kernels (the pixel-word and the
 * row-run ones; frame groups in flight from 8 up to the resident capacity)
 * on scratch frames with a scratch keystream, and set the fastest with
 * cv_key_set_launch (the key's path becomes CV_PATH_FUSED; its generator
 * state does not change).  With CV_TUNE_CACHE naming a file, the winner is
 * stored there under the key's geometry, direction and n_frames, and a later
 * call for the same class takes it from the file without timing (*cached =
 * 1).  `best` (may be NULL) receives the launch shape.  Errors: CV_E_INVAL
 * (NULL key, n_frames = 0, geometry without the pixel-word conditions),
 * CV_E_NOMEM, CV_E_HIP. */
cv_status cv_key_autotune(cv_key *key, int decrypt, uint32_t n_frames, void *stream,
                          cv_launch *best, int *cached);

/* Graphs captured and replayed by the key's calls since its set-up
 * (cv_launch.use_graph).  Errors: CV_E_INVAL (NULL). */
cv_status cv_key_graph_counts(const cv_key *key, uint64_t *captures, uint64_t *replays);

/* Internal batches that took the lookahead's keystream, and lookaheads
 * dropped because the next batch differed (cv_launch.lookahead).  Errors:
 * CV_E_INVAL (NULL). */
cv_status cv_key_lookahead_counts(const cv_key *key, uint64_t *hits, uint64_t *misses);

/* Choose the round implementation (CV_PATH_*).  CV_E_INVAL if unknown. */
cv_status cv_key_set_path(cv_key *key, int path);

/* Read the key's launch shape (chosen at cv_keysetup from the geometry and
 * the device's LDS size). */
cv_status cv_key_get_launch(const cv_key *key, cv_launch *launch);

/* Set the launch shape (drops the key's captured graphs).  CV_E_INVAL if
 * batch_frames = 0, use_graph > 1, threads is not a
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
 *  s_c       host array of n_frames confusion seeds (Algorithm 1 draws one
 *            per frame), each >= 1.
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
 * r*floor(i*H/n)*W*C) and advance the key (Algorithm 2: each subframe's
 * generator runs until the frame's bytes of that subframe exist).
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

/* Size of the static device scratch of cv_apply_rounds_noalloc (per device). */
#define CV_NOALLOC_SCRATCH_BYTES (64u << 20)

/* cv_apply_rounds for callers that cannot allocate device memory (code that
 * must not call hipMalloc, such as a tight serving loop or a harness that
 * forbids it): the same arguments, rounds and bytes, but every buffer the
 * kernels need beyond the caller's frames and keystream -- shift tables,
 * exchange frames and barrier counters of the fused kernels, the byte
 * kernels' ping-pong frames, the error word -- lives in one static device
 * array of CV_NOALLOC_SCRATCH_BYTES that each device the library runs on
 * holds until the process ends.  The call allocates nothing (no hipMalloc,
 * hipHostMalloc or event), whatever the key's workspace holds; it runs the
 * fused kernels when the pixel-word conditions hold (see CV_PATH_FUSED),
 * else the byte kernels, in chunks of frames that fit the scratch.
 * Synchronous: it returns when its frames are done (the shift tables go up
 * from a static host array, a copy the runtime performs synchronously).
 * Calls are serialised within the process; calls that overlap on one GPU
 * from different copies of the library would race on its scratch.
 * Errors: as cv_apply_rounds; CV_E_INVAL if even one frame does not fit the
 * scratch (fused kernels: two pixel-word frames of 4*H*W bytes plus one
 * shift table of 4*H bytes; byte kernels: one frame plus its shift table;
 * H at most 262144), with a message naming the limit; CV_E_HIP if a group
 * barrier timed out, in which case this call's output frames are invalid
 * (the error word is cleared at the start of every call, and the key is not
 * affected). */
cv_status cv_apply_rounds_noalloc(cv_key *key, int decrypt, const uint8_t *in, uint8_t *out,
                                  const uint8_t *ks, const uint32_t *s_c, size_t n_frames,
                                  void *stream);

/* ------------------------------------------------------------------------
 * Many streams per tick.  A batch object runs one tick of several video
 * streams -- each with its own key, resolution and number of subframes --
 * as one keystream launch over the band generators of all streams and one
 * persistent rounds launch over all (stream, frame) jobs, instead of one
 * pair of launches per stream.  This is Algorithm 1 (one master splitting
 * every frame into subframes handled in parallel, Algorithm 2 per subframe)
 * applied to many streams at once: a frame job is handled by a group of G
 * workgroups on one XCD, band b by workgroup b mod G, with a group barrier
 * between rounds (Sec. 2's round structure: every band of round j is
 * diffused before any band of round j+1 is confused).
 *
 * The bytes written are identical to cv_encrypt_frames / cv_decrypt_frames
 * on each item's key.  Items whose geometry or buffers do not meet the
 * pixel-word conditions (C in {3,4}, W % 16 == 0, 16-byte aligned in/out)
 * run on their key's own path within the same call, in stream order.
 */
typedef struct cv_batch cv_batch;

/* One stream's share of a tick. */
typedef struct {
  cv_key *key;          /* the stream's key; advances by n_frames frames; at most once per tick */
  const uint8_t *in;    /* device, n_frames*H*W*C bytes (HWC frames back to back) */
  uint8_t *out;         /* device, same size; overlaps no other buffer of the tick */
  const uint32_t *s_c;  /* host, n_frames confusion seeds, each >= 1 */
  uint32_t n_frames;    /* 0 = the item is skipped */
  int32_t decrypt;      /* 0: encrypt (Eq. 1 then Eq. 3 per round); 1: decrypt (Eq. 4 then Eq. 2) */
} cv_batch_item;

/* Launch shape of the batched rounds kernel; any shape gives the same bytes. */
typedef struct {
  uint32_t threads;     /* threads per workgroup: 256..1024, multiple of 64.  With 1024, a
                           channel count's jobs run on the row-run kernel (encryption by
                           whole source-row runs, decryption in one pass per tile) when
                           every one of them has tiles that fit the LDS; otherwise, and
                           with fewer threads, on the pixel-word kernel */
  uint32_t group_wgs;   /* G, workgroups per frame job: 1..64.  With max_groups = 0 the
                           planner may also form larger groups (multiples of G, up to the
                           workgroups of one XCD) for frames with more than G subframes,
                           when that shortens the tick by its cost model (rounds x
                           ceil(n / group size) x band rows x W per job, longest job first
                           onto the group where it finishes first) */
  uint32_t max_groups;  /* frame jobs in flight at once, in groups of exactly G; 0 = as many
                           as can be resident */
  uint32_t use_graph;   /* 1: capture a tick in a HIP graph and replay it while the tick's
                           structure (items' geometries, frame counts and launch sizes) is
                           unchanged; 0: launch kernel by kernel */
  uint32_t tile_rows_max; /* frame rows per LDS tile at most (the LDS tiling); 0 = as many
                           as fit */
  uint32_t prefetch;    /* 1: once a tick's keystream is generated, generate the next tick's
                           -- the same keys and frame counts, one tick on -- on a private
                           stream while this tick's rounds run (on compute units the rounds
                           leave free for it when the device is still busy with earlier
                           ticks), from a copy of the keys' generator states made
                           on the tick's stream (the keystream depends only on them,
                           Algorithm 2).  The next cv_batch_run takes it when its batched
                           items are the same keys (any order) at the frame index and frame
                           count predicted, copying the advanced states into the keys on its
                           stream; otherwise it generates its own keystream and the
                           prefetched work is dropped.  The private stream never touches a
                           key; it is chosen as for cv_launch.lookahead (its own hardware
                           queue beside a stream other than the null stream, non-blocking
                           beside the null stream).  Ticks then go kernel by kernel,
                           without graphs.  0: off */
} cv_batch_shape;

/* Counters of a batch object (host-side, no synchronisation). */
typedef struct {
  uint64_t ticks;               /* cv_batch_run calls that enqueued work */
  uint64_t graph_captures;      /* ticks that captured a new graph */
  uint64_t graph_replays;       /* ticks that replayed a captured graph */
  uint32_t last_jobs;           /* frame jobs of the last tick on the batched kernels */
  uint32_t last_groups;         /* groups in flight in the last tick's rounds launches */
  uint32_t last_chains;         /* band generators of the last tick's keystream launches */
  uint32_t last_fallback_items; /* items of the last tick that ran on their key's own path */
  uint32_t tune_cache_hits;     /* cv_batch_autotune calls answered from CV_TUNE_CACHE */
  uint32_t tune_shapes_timed;   /* launch shapes the autotuner timed */
  uint32_t prefetch_hits;       /* ticks that took a prefetched keystream */
  uint32_t prefetch_misses;     /* prefetched keystreams dropped (the next tick differed) */
  uint32_t last_wide_groups;    /* groups of the last tick larger than group_wgs */
} cv_batch_info;

/* Create a batch object on HIP device `device` (the keys of its items must
 * live there).  Default shape: 1024 threads, G = 8, resident capacity,
 * graphs on, largest tiles, prefetch on.  Errors: CV_E_INVAL (NULL, no such
 * device), CV_E_NOMEM. */
cv_status cv_batch_create(int device, cv_batch **out);

/* Release a batch object (synchronises its device).  NULL is ignored.  The
 * keys of its items are not touched. */
void cv_batch_free(cv_batch *batch);

cv_status cv_batch_get_shape(const cv_batch *batch, cv_batch_shape *shape);

/* CV_E_INVAL if threads or group_wgs is out of range or use_graph or
 * prefetch > 1. */
cv_status cv_batch_set_shape(cv_batch *batch, const cv_batch_shape *shape);

/* Encrypt or decrypt one tick: every item's n_frames frames, with keystream
 * generation and r rounds (Algorithms 1-2), on `stream`.  The whole tick is
 * checked before anything is enqueued: on error no key advances.  Errors:
 * CV_E_INVAL (NULL pointers with n_frames > 0, a key twice, a key on
 * another device, an s_c of 0, overlapping buffers), CV_E_NOMEM, CV_E_HIP
 * (including a group barrier timeout of an earlier tick, which leaves that
 * tick's output invalid and every later call on this batch failing).
 * Calls on one batch are ordered with each other even across streams.
 * Items the batched kernels do not take -- 2DLASM keys, geometries outside
 * C in {3,4} with W a multiple of 16, unaligned buffers -- run on their
 * key's own path, one after another on `stream`
 * (cv_batch_info.last_fallback_items). */
cv_status cv_batch_run(cv_batch *batch, const cv_batch_item *items, size_t n_items,
                       void *stream);

/* Wait for the batch's last tick and report its asynchronous errors. */
cv_status cv_batch_sync(cv_batch *batch);

cv_status cv_batch_get_info(const cv_batch *batch, cv_batch_info *info);

/* Time the rounds kernel of the tick `items` describes for candidate shapes
 * and keep the fastest: the kernel (threads 512: pixel-word; 1024: row-run
 * where it applies), the band-to-workgroup mapping G in {4, 8, 16, 32}, the
 * groups in flight (all resident, or half), and the LDS tiling (the largest
 * tiles that fit, or half as many rows).  With the environment variable
 * CV_TUNE_CACHE naming a file, the winner is stored there under the tick's
 * shape class (its items' geometries, directions and frame counts) and a
 * later call for the same class takes it from the file without timing
 * (cv_batch_info.tune_cache_hits).  Keys are not advanced and no keystream
 * is generated: the out buffers of the items receive meaningless bytes.
 * `best` (may be NULL) receives the chosen shape.  Same argument errors as
 * cv_batch_run. */
cv_status cv_batch_autotune(cv_batch *batch, const cv_batch_item *items, size_t n_items,
                            void *stream, cv_batch_shape *best);

/* Event timing of the batch's keystream and rounds launches while on (the
 * totals use cv_profile's fields; round_frames counts frame-rounds).  With
 * profiling on, ticks are launched kernel by kernel, not as graphs. */
cv_status cv_batch_set_profiling(cv_batch *batch, int on);
cv_status cv_batch_get_profile(cv_batch *batch, cv_profile *prof);

/* ------------------------------------------------------------------------
 * Serving.  A server owns a worker thread that runs many live video streams
 * on one device: every stream keeps a ring of keystream frames generated
 * ahead of its frames' arrival (the keystream depends only on the key
 * state, Algorithm 2), and frames submitted by any stream are collected
 * into ticks of the batched rounds kernel as soon as their keystream is
 * ready (continuous batching).  A frame's latency is then the wait for the
 * next tick plus the r rounds, not the sequential generator chain.  The
 * real-time criterion of the paper is 24 frames per second per stream.
 *
 * Streams are admitted while the server's device-memory budget holds their
 * keystream rings (ring_frames * r*H*W*C bytes each); frame and output
 * buffers are the caller's.  The bytes of every frame are identical to
 * cv_encrypt_frames / cv_decrypt_frames on a key built from the same p_m.
 */
typedef struct cv_server cv_server;
typedef struct cv_stream cv_stream;

/* Start a server on `device`.  hbm_budget > 0: that many bytes of device
 * memory for keystream rings, allocated now; a stream is admitted while
 * they hold its ring.  hbm_budget = 0: rings are allocated as streams open,
 * in chunks of at least 4 GiB, and a stream is admitted while the device's
 * free memory at that moment, less a reserve of a sixteenth of the total,
 * holds its ring (cv_server_stats.hbm_budget then reports the chunks taken
 * so far).  Ring depth 3 frames and 8 queued frames per stream unless
 * cv_server_tune says otherwise.  Errors: CV_E_INVAL (NULL, no such
 * device), CV_E_NOMEM. */
cv_status cv_server_create(int device, size_t hbm_budget, cv_server **out);

/* Ring depth (keystream frames generated ahead, >= 1) and queue depth
 * (frames a stream may have submitted and not finished, >= 1) for streams
 * opened after the call.  A deeper ring lets a stream's generator run
 * further ahead while arrivals are few, which absorbs bursts of arrivals
 * near the generator's serial rate (ring_frames * r*H*W*C bytes of device
 * memory per stream).  split_cus = q in 1..3 runs keystream generation
 * on q quarters of the compute units of every XCD and the rounds on the
 * rest (1, a quarter, is the default); 0 lets both use every CU.
 * CV_E_INVAL if a depth is 0 or above 64 or split_cus is outside 0..3;
 * CV_E_STATE if split_cus changes while streams are open. */
cv_status cv_server_tune(cv_server *server, uint32_t ring_frames, uint32_t queue_frames,
                         int split_cus);

/* Stop the worker after the submitted frames are done, close every stream
 * and release the server.  NULL is ignored. */
void cv_server_free(cv_server *server);

/* Block until every submitted frame of every stream is done.  Returns the
 * error that stopped the server, if any. */
cv_status cv_server_drain(cv_server *server);

typedef struct {
  uint64_t frames_done;         /* frames whose rounds have completed */
  uint64_t rounds_ticks;        /* batched rounds launches */
  uint64_t keystream_launches;  /* keystream generation launches */
  uint64_t keystream_frames;    /* stream-frames of keystream generated */
  uint32_t open_streams;
  uint32_t split_cus;           /* quarters of every XCD's CUs that keystream generation
                                    runs on, apart from the rounds (0: CUs shared) */
  uint64_t hbm_used, hbm_budget; /* keystream ring bytes in use / held (the fixed budget, or
                                    the chunks taken so far when it grows) */
  double keystream_ms;          /* summed launch-to-completion time of keystream launches */
  double rounds_ms;             /* summed launch-to-completion time of rounds ticks */
  uint64_t starved_frames;      /* frames that waited in the queue for their keystream */
} cv_server_stats;

cv_status cv_server_get_stats(cv_server *server, cv_server_stats *stats);

/* Open a stream (one direction: decrypt = 0 encrypts, 1 decrypts) with its
 * own key (same geometry, map and p_m rules and errors as cv_keysetup).
 * Keystream generation for its first frames starts at once.  CV_E_AGAIN
 * if the budget cannot hold its ring or 4096 streams are open. */
cv_status cv_stream_open(cv_server *server, const cv_geom *geom, cv_map map, const double *p_m,
                         size_t n_doubles, int decrypt, cv_stream **out);

/* Queue the stream's next frame: `frame` and `out` are device buffers of
 * H*W*C bytes that must stay valid, and not be written, until the frame is
 * done; `out` must not overlap another frame buffer in flight.  s_c >= 1
 * is the frame's confusion seed.  *ticket receives the frame's number in
 * the stream (0, 1, 2, ...).  CV_E_AGAIN if queue_frames frames are in
 * flight; CV_E_INVAL for NULL buffers, frame == out or s_c = 0; CV_E_HIP
 * if the server stopped on an error. */
cv_status cv_stream_submit(cv_stream *stream, const uint8_t *frame, uint8_t *out, uint32_t s_c,
                           uint64_t *ticket);

/* *done = 1 once frame `ticket` is in its output buffer; *latency_ms (may
 * be NULL) then receives the time from its submission to the worker seeing
 * its tick complete (or -1 for tickets more than 4096 frames old).
 * CV_E_INVAL for a ticket not yet issued. */
cv_status cv_stream_poll(cv_stream *stream, uint64_t ticket, int *done, double *latency_ms);

/* Wait for the stream's frames, then release the stream and its key. */
cv_status cv_stream_close(cv_stream *stream);

#ifdef __cplusplus
}
#endif

#endif /* CHAOSVID_H */
