// Host runtime and C ABI of libchaosvid (declarations and contract in
// include/chaosvid.h).
//
// A key owns the device-resident generator state of one stream and the
// workspace its calls reuse: keystream for a batch of frames, one scratch
// frame buffer per batch frame (the rounds ping-pong between it and the
// output), and the per-frame row-shift tables.  Work is cut into batches of
// at most `batch_frames` frames; per batch: shift tables H2D, one PRBG launch
// for the whole batch, then r round launches over the whole batch.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <cmath>

#include <algorithm>
#include <atomic>
#include <mutex>
#include <string>
#include <vector>

#include "runtime.h"


namespace cv {
namespace rt {

thread_local std::string g_last_error;

hipError_t copy_sync(void* dst, const void* src, size_t bytes, hipMemcpyKind kind);

cv_status fail(cv_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

cv_status hip_fail(hipError_t e, const char* what) {
  return fail(CV_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}



// Sec. 2, Eq. (1): g(alpha) = floor(s_c * sin((2*pi*alpha)/H)), binary64,
// left to right, reduced mod W for the kernels (beta = (o + g) mod W).
void shift_table(uint32_t H, uint32_t W, uint32_t s_c, uint32_t* gm) {
#pragma clang loop vectorize(disable)
  for (uint32_t alpha = 0; alpha < H; alpha++) {
    const double angle = ((2.0 * M_PI) * (double)alpha) / (double)H;
    const int64_t g = (int64_t)floor((double)s_c * sin(angle));
    int64_t m = g % (int64_t)W;
    if (m < 0) m += W;
    gm[alpha] = (uint32_t)m;
  }
}

hipEvent_t pooled_event(cv_key* k) {
  if (!k->event_pool.empty()) {
    hipEvent_t e = k->event_pool.back();
    k->event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Fold finished spans into the totals and recycle their events.
cv_status drain_spans(cv_key* k) {
  for (auto& sp : k->spans) {
    CV_HIP(hipEventSynchronize(sp.b));
    float ms = 0.f;
    CV_HIP(hipEventElapsedTime(&ms, sp.a, sp.b));
    if (sp.kind == 0) {
      k->prof.prbg_ms += ms;
      k->prof.prbg_launches++;
      k->prof.prbg_steps += sp.work;
    } else {
      k->prof.round_ms += ms;
      k->prof.round_launches++;
      k->prof.round_frames += sp.work;
    }
    k->event_pool.push_back(sp.a);
    k->event_pool.push_back(sp.b);
  }
  k->spans.clear();
  return CV_OK;
}

// Optional events around one launch: begin() before, end() after.
struct Timed {
  cv_key* k;
  hipStream_t st;
  hipEvent_t a = nullptr;
  Timed(cv_key* key, hipStream_t s) : k(key), st(s) {
    if (k && k->profiling && (a = pooled_event(k)) != nullptr) (void)hipEventRecord(a, st);
  }
  void end(int kind, uint64_t work) {
    if (!a) return;
    hipEvent_t b = pooled_event(k);
    if (!b) return;
    (void)hipEventRecord(b, st);
    k->spans.push_back({a, b, kind, work});
    if (k->spans.size() > 4096) (void)drain_spans(k);
  }
};

// Generator variant for the next launch: the requested one, or the IEEE
// division when the key is outside the reciprocal division's domain.
int prbg_variant(const cv_key* k) {
  if (!k->fast || k->prbg_variant == 1) return cv::PRBG_EXACT;
  if (k->prbg_variant == 2) return cv::PRBG_RECIP;
  if (k->prbg_variant == 3) return cv::PRBG_RECIP_PAIR;
  if (k->prbg_variant == 5) return cv::PRBG_SPEC_PLANT;
  return cv::PRBG_SPEC;
}

uint64_t prbg_steps(const cv_key* k, uint64_t frames) {
  uint64_t steps = 0;
  const uint64_t row = (uint64_t)k->g.W * k->g.C;
  const uint64_t per_step = k->map == CV_MAP_2DLASM ? 12 : 6;  // keystream bytes per step
  for (uint32_t i = 0; i < k->g.n; i++) {
    const uint64_t S = (cv::band_lo(k->g.H, k->g.n, i + 1) - cv::band_lo(k->g.H, k->g.n, i)) * row;
    steps += (k->g.r * S + per_step - 1) / per_step;
  }
  return steps * frames;
}

// Keystream of T frames into ks (layout of cv_keystream_frames) on st,
// advancing the key's generators.
cv_status launch_keystream(cv_key* k, uint8_t* ks, uint32_t T, hipStream_t st) {
  Timed tm(k, st);
  if (k->map == CV_MAP_2DLASM) {
    CV_HIP(cv::launch_prbg_lasm(k->d_lchains, k->g.n, ks, T, 0, k->d_err, st));
    tm.end(0, prbg_steps(k, T));
    return queue_err_readback(k, st);
  }
  CV_HIP(cv::launch_prbg_plcm(k->d_chains, k->g.n, ks, T, prbg_variant(k), st));
  tm.end(0, prbg_steps(k, T));
  return CV_OK;
}

// Largest pixel-word tile (rows) not above `want` that the kernels accept
// with `threads` threads: every (row, run) pair of a gather gets a thread
// (rows * ceil(W/H) <= threads) and the diffusion pass gives each thread 16
// pixels (rows * W <= 16 * threads).
uint32_t pw_tile_limit(const Geom& g, uint32_t threads, uint32_t want) {
  const uint32_t M = (g.W + g.H - 1) / g.H;
  uint32_t t = std::min(want, threads / M);
  t = std::min<uint64_t>(t, (16ull * threads) / g.W);
  return std::min(t, g.H);
}

uint32_t pw_tile_rows(const Geom& g, uint32_t threads, size_t lds_max) {
  const size_t budget = std::min<size_t>(lds_max, 64 * 1024);
  uint32_t rows = 0;
  while (rows < g.H && cv::round_pw_lds_bytes(g, rows + 1) <= budget) rows++;
  return pw_tile_limit(g, threads, rows);
}

size_t lds_limit(int device) {
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) return 64 * 1024;
  return prop.sharedMemPerBlock;
}

bool ranges_overlap(const void* a, size_t na, const void* b, size_t nb) {
  const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
  return x < y + nb && y < x + na;
}

// Executable graphs reference the key's workspace and launch shape: drop
// them whenever either changes (waits for the device first, since a graph
// may still be running).
void drop_graphs(cv_key* k) {
  if (k->graphs.empty()) return;
  (void)hipDeviceSynchronize();
  for (auto& g : k->graphs) (void)hipGraphExecDestroy(g.exec);
  k->graphs.clear();
}

void free_workspace(cv_key* k) {
  drop_graphs(k);
  if (k->d_ks) (void)hipFree(k->d_ks);
  if (k->d_scratch) (void)hipFree(k->d_scratch);
  if (k->d_scratch2) (void)hipFree(k->d_scratch2);
  k->d_scratch2 = nullptr;
  if (k->d_gm) (void)hipFree(k->d_gm);
  if (k->h_gm) (void)hipHostFree(k->h_gm);
  k->d_ks = k->d_scratch = nullptr;
  k->d_gm = nullptr;
  k->h_gm = nullptr;
  k->ws_frames = 0;
}

cv_status ensure_workspace(cv_key* k, size_t frames) {
  if (frames <= k->ws_frames) return CV_OK;
  if (k->gm_pending) {
    CV_HIP(hipEventSynchronize(k->gm_done));
    k->gm_pending = false;
  }
  CV_HIP(hipDeviceSynchronize());  // older buffers may still be in use
  free_workspace(k);
  const Geom& g = k->g;
  const uint64_t scratch = std::max<uint64_t>(k->F, (uint64_t)g.H * g.W * 4);
  if (hipMalloc(&k->d_ks, frames * (uint64_t)g.r * k->F) != hipSuccess ||
      hipMalloc(&k->d_scratch, frames * scratch) != hipSuccess ||
      hipMalloc(&k->d_scratch2, frames * scratch) != hipSuccess ||
      hipMalloc(&k->d_gm, frames * (uint64_t)g.H * sizeof(uint32_t)) != hipSuccess ||
      hipHostMalloc(&k->h_gm, frames * (uint64_t)g.H * sizeof(uint32_t)) != hipSuccess) {
    (void)hipGetLastError();
    free_workspace(k);
    return fail(CV_E_NOMEM, "workspace allocation failed");
  }
  k->ws_frames = frames;
  return CV_OK;
}

// Stage the shift tables of `T` frames and copy them to the device.
cv_status upload_shift_tables(cv_key* k, const uint32_t* s_c, size_t T, hipStream_t st) {
  if (k->gm_pending) {  // the staging buffer is still being read by an earlier copy
    CV_HIP(hipEventSynchronize(k->gm_done));
    k->gm_pending = false;
  }
  const Geom& g = k->g;
  for (size_t t = 0; t < T; t++) shift_table(g.H, g.W, s_c[t], k->h_gm + t * g.H);
  CV_HIP(hipMemcpyAsync(k->d_gm, k->h_gm, T * g.H * sizeof(uint32_t), hipMemcpyHostToDevice, st));
  CV_HIP(hipEventRecord(k->gm_done, st));
  k->gm_pending = true;
  return CV_OK;
}

cv::RoundArgs round_args(const cv_key* k, const uint8_t* ks, uint32_t T) {
  cv::RoundArgs a{};
  a.ks = ks;
  a.gm = k->d_gm;
  a.frame_bytes = k->F;
  a.ks_stride = (uint64_t)k->g.r * k->F;
  a.g = k->g;
  a.n_frames = T;
  return a;
}

// r rounds over T frames (keystream already in `ks`).  Round outputs
// alternate between `out` and the scratch buffer so that the last round
// lands in `out` and no round reads the buffer it writes.
bool aligned16(const void* p) { return ((uintptr_t)p & 15u) == 0; }

// A device-side error (a fused launch that timed out at a group barrier or
// found a group spread over XCDs, a 2DLASM sine that could not be rounded)
// leaves the key's error word set.  It is reported (CV_E_HIP) by the first
// call that finds the word's read-back complete -- every call when `wait` --
// and from then on the key is dead: every later call fails with CV_E_STATE.
// The word itself is never cleared, so the kernels of a dead key that were
// already queued give up at once instead of producing more output.
cv_status check_async_errors(cv_key* k, bool wait) {
  if (k->dead) return fail(CV_E_STATE, "the key is unusable after an earlier device error (" +
                                           k->dead_msg + "); free it and set up a new key");
  if (!k->err_pending) return CV_OK;
  if (wait) {
    CV_HIP(hipEventSynchronize(k->err_copied));
  } else if (hipEventQuery(k->err_copied) != hipSuccess) {
    (void)hipGetLastError();
    return CV_OK;
  }
  k->err_pending = false;
  if (*k->h_err) {
    k->dead = true;
    k->dead_msg = *k->h_err == 2
                      ? "a 2DLASM sine could not be rounded with certainty; the keystream and "
                        "the generator state are invalid"
                      : "a fused launch timed out at a group barrier or found a group spread "
                        "over XCDs; its output is invalid";
    return fail(CV_E_HIP, k->dead_msg);
  }
  return CV_OK;
}

// Resident capacity of the fused kernel for the key's shape, and the number of
// groups to use (`want` rounded down to a multiple of 8, 0 = capacity).
void set_fused_groups(cv_key* k, uint32_t want) {
  const Geom& g = k->g;
  k->fused_cap = 0;
  if (k->tile_pw > 0 && (g.C == 3 || g.C == 4) && g.W % 16 == 0)
    k->fused_cap = cv::rounds_fused_resident_groups(g, k->tile_pw, k->threads, k->device);
  k->tile_skew = cv::rounds_skew_tile_rows(g, k->lds_max);
  k->fused_cap_skew = cv::rounds_skew_resident_groups(g, k->tile_skew, k->device);
  k->fused_cap_unskew = cv::rounds_unskew_applies(g, k->lds_max)
                            ? cv::rounds_unskew_resident_groups(g, k->device) : 0;
  k->rows_tile_dec = k->rows_G = k->fused_cap_rows = 0;
  if (k->fused_cap_unskew == 0 && k->tile_skew > 0) {
    const uint32_t tile = cv::batch_unskew_tile_rows(g, k->lds_max);
    const size_t lds = cv::batch_rows_lds_bytes(g, true, tile);
    const uint32_t kq = g.W % 12 == 0 ? 12 : 4;
    const uint32_t per_xcd =
        tile > 0 ? cv::batch_resident_slots(g.C, kq, true, 1024, lds, k->device) : 0;
    if (per_xcd > 0) {
      k->rows_tile_dec = tile;
      k->rows_lds = lds;
      k->rows_KQ = kq;
      k->rows_G = std::min(g.n, per_xcd);
      k->fused_cap_rows = 8 * (per_xcd / k->rows_G);
    }
  }
  const uint32_t w = want / 8 * 8;
  k->fused_groups = (w == 0 || w > k->fused_cap) ? k->fused_cap : w;
}

// The key's asynchronous error word (a fused launch's barrier timeout, a
// 2DLASM sine that could not be rounded) and its pinned read-back.
cv_status ensure_err_flag(cv_key* k) {
  if (k->d_err) return CV_OK;
  if (hipMalloc(&k->d_err, sizeof(uint32_t)) != hipSuccess ||
      hipHostMalloc(&k->h_err, sizeof(uint32_t)) != hipSuccess) {
    (void)hipGetLastError();
    return fail(CV_E_NOMEM, "error-flag allocation failed");
  }
  *k->h_err = 0;
  const uint32_t zero = 0;
  CV_HIP(copy_sync(k->d_err, &zero, sizeof(zero), hipMemcpyHostToDevice));
  CV_HIP(hipEventCreateWithFlags(&k->err_copied, hipEventDisableTiming));
  return CV_OK;
}

// Bring the error word back to the host behind the work just enqueued on st;
// the next call on the key reports it.
cv_status queue_err_readback(cv_key* k, hipStream_t st) {
  CV_HIP(hipMemcpyAsync(k->h_err, k->d_err, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
  if (k->capturing) {  // the event is recorded after each replay instead
    k->captured_err = true;
    return CV_OK;
  }
  CV_HIP(hipEventRecord(k->err_copied, st));
  k->err_pending = true;
  return CV_OK;
}

cv_status ensure_fused(cv_key* k) {
  if (k->d_fscratch) return CV_OK;
  const Geom& g = k->g;
  const uint64_t pwf = (uint64_t)g.H * g.W * 4;
  if (hipMalloc(&k->d_fscratch, (uint64_t)k->fused_groups * 2 * pwf) != hipSuccess ||
      hipMalloc(&k->d_counters, 128ull * k->fused_groups) != hipSuccess) {
    (void)hipGetLastError();
    k->d_fscratch = nullptr;
    return fail(CV_E_NOMEM, "fused-path workspace allocation failed");
  }
  return ensure_err_flag(k);
}

// Fused kernel of a direction: the row-run kernels (encryption: any
// geometry with the pixel-word conditions; decryption: every band one LDS
// tile) unless the pixel-word kernels are asked for.
// Decryption of geometries with a band over one LDS tile takes the row-run
// batch kernel (tile by tile) over the key's frames.
enum FusedKernel { FUSED_PW = 0, FUSED_SKEW = 1, FUSED_UNSKEW = 2, FUSED_ROWS = 3 };

FusedKernel fused_kernel(const cv_key* k, bool decrypt) {
  if (k->round_variant == 2) return FUSED_PW;
  if (!decrypt) return k->fused_cap_skew > 0 ? FUSED_SKEW : FUSED_PW;
  if (k->fused_cap_unskew > 0) return FUSED_UNSKEW;
  return k->fused_cap_rows > 0 ? FUSED_ROWS : FUSED_PW;
}

uint32_t fused_group_cap(const cv_key* k, bool decrypt) {
  switch (fused_kernel(k, decrypt)) {
    case FUSED_SKEW: return std::min(k->fused_groups, k->fused_cap_skew);
    case FUSED_UNSKEW: return std::min(k->fused_groups, k->fused_cap_unskew);
    case FUSED_ROWS: return std::min(k->fused_groups, k->fused_cap_rows);
    default: return k->fused_groups;
  }
}

// Tables of the row-run batch kernel for up to T frames (decryption with
// FUSED_ROWS); nothing to do for other keys.
cv_status ensure_rows_tables(cv_key* k, uint32_t T) {
  if (k->fused_cap_rows == 0) return CV_OK;
  const size_t bytes =
      cv::stream_rows_table_bytes(T, cv::stream_rows_slots(k->fused_cap_rows, k->rows_G));
  if (bytes <= k->rows_tables_cap) return CV_OK;
  drop_graphs(k);                  // captured launches point at the old tables
  CV_HIP(hipDeviceSynchronize());  // which may still be read
  if (k->d_rows_tables) (void)hipFree(k->d_rows_tables);
  k->d_rows_tables = nullptr;
  k->rows_tables_cap = 0;
  if (hipMalloc(&k->d_rows_tables, bytes) != hipSuccess) {
    (void)hipGetLastError();
    k->d_rows_tables = nullptr;
    return fail(CV_E_NOMEM, "row-run decryption tables allocation failed");
  }
  k->rows_tables_cap = bytes;
  return CV_OK;
}

// One fused launch over T frames with the workspace given explicitly: shift
// tables `gm`, two pixel-word frames per group in `fscratch`, 128 bytes per
// group in `counters`, the error word `err`; at most `groups` groups.
cv_status launch_fused_ws(const cv_key* k, bool decrypt, const uint8_t* in, uint8_t* out,
                          const uint8_t* ks, uint32_t T, const uint32_t* gm, uint8_t* fscratch,
                          uint32_t* counters, uint32_t* err, uint32_t groups, hipStream_t st,
                          uint8_t* rows_tables) {
  cv::RoundsFusedArgs a{};
  a.in = in;
  a.out = out;
  a.ks = ks;
  a.gm = gm;
  a.scratch = fscratch;
  a.counters = counters;
  a.err = err;
  a.g = k->g;
  a.tile_rows = k->tile_pw;
  a.n_frames = T;
  a.groups = std::min<uint32_t>(std::min(groups, fused_group_cap(k, decrypt)), ((T + 7) / 8) * 8);
  a.spin_limit = k->spin_limit;
  a.decrypt = decrypt;
  FusedKernel fk = fused_kernel(k, decrypt);
  if (fk == FUSED_ROWS && !rows_tables) fk = FUSED_PW;
  switch (fk) {
    case FUSED_SKEW: CV_HIP(cv::launch_rounds_skew(a, k->tile_skew, st)); break;
    case FUSED_UNSKEW: CV_HIP(cv::launch_rounds_unskew(a, st)); break;
    case FUSED_ROWS: {
      cv::StreamRows r{};
      r.proto.in = in;
      r.proto.out = out;
      r.proto.in_last = in + (uint64_t)T * k->F - 4;
      r.proto.ks = ks;
      r.proto.gm = gm;
      r.proto.g = k->g;
      r.proto.decrypt = 1;
      r.proto.tile_dec = k->rows_tile_dec;
      r.ks_stride = (uint64_t)k->g.r * k->F;
      r.T = T;
      r.groups = a.groups;
      r.G = k->rows_G;
      r.KQ = k->rows_KQ;
      r.lds = k->rows_lds;
      r.tables = rows_tables;
      r.scratch = fscratch;
      r.counters = counters;
      r.err = err;
      r.spin_limit = k->spin_limit;
      CV_HIP(cv::launch_stream_rows(r, st));
      break;
    }
    default: CV_HIP(cv::launch_rounds_fused(a, k->threads, st));
  }
  return CV_OK;
}

cv_status run_rounds_fused(cv_key* k, bool decrypt, const uint8_t* in, uint8_t* out,
                           const uint8_t* ks, uint32_t T, hipStream_t st) {
  cv_status s = ensure_fused(k);
  if (s == CV_OK && decrypt) s = ensure_rows_tables(k, T);
  if (s != CV_OK) return s;
  Timed tm(k, st);
  if ((s = launch_fused_ws(k, decrypt, in, out, ks, T, k->d_gm, k->d_fscratch, k->d_counters,
                           k->d_err, k->fused_groups, st, k->d_rows_tables)) != CV_OK)
    return s;
  tm.end(1, (uint64_t)T * k->g.r);
  return queue_err_readback(k, st);
}

bool pw_eligible(const cv_key* k, const uint8_t* in, const uint8_t* out, uint32_t threads,
                 size_t lds_max) {
  const Geom& g = k->g;
  if (!((g.C == 3 || g.C == 4) && g.W % 16 == 0 && aligned16(in) && aligned16(out))) return false;
  const uint32_t t = pw_tile_rows(g, threads, lds_max);
  return t > 0 && cv::round_pw_lds_bytes(g, t) <= lds_max;
}

// Pixel-word kernels apply: 3 or 4 channels, 16-byte rows and buffers.
bool use_pw(const cv_key* k, const uint8_t* in, const uint8_t* out, const uint8_t* ks) {
  if (k->round_variant == 1) return false;
  const Geom& g = k->g;
  return (g.C == 3 || g.C == 4) && g.W % 16 == 0 && aligned16(in) &&
         aligned16(out) && aligned16(ks) && k->tile_pw > 0;
}

cv_status run_rounds_pw(cv_key* k, bool decrypt, const uint8_t* in, uint8_t* out,
                        const uint8_t* ks, uint32_t T, hipStream_t st) {
  const uint32_t r = k->g.r;
  cv::RoundPwArgs a{};
  a.ks = ks;
  a.gm = k->d_gm;
  a.g = k->g;
  a.n_frames = T;
  a.tile_rows = k->tile_pw;
  a.decrypt = decrypt;
  const uint8_t* cur = in;
  for (uint32_t s = 0; s < r; s++) {
    const bool last = s + 1 == r;
    uint8_t* target = last ? out : (s % 2 == 0 ? k->d_scratch : k->d_scratch2);
    a.src = cur;
    a.dst = target;
    a.src_packed = s == 0;
    a.dst_packed = last;
    a.j = decrypt ? r - 1 - s : s;
    Timed tm(k, st);
    CV_HIP(cv::launch_round_pw(a, k->threads, st));
    tm.end(1, T);  // T frame-rounds
    cur = target;
  }
  return CV_OK;
}

cv_status run_rounds(cv_key* k, bool decrypt, const uint8_t* in, uint8_t* out, const uint8_t* ks,
                     uint32_t T, hipStream_t st) {
  if (use_pw(k, in, out, ks)) {
    if (k->path == CV_PATH_FUSED && k->fused_groups > 0)
      return run_rounds_fused(k, decrypt, in, out, ks, T, st);
    return run_rounds_pw(k, decrypt, in, out, ks, T, st);
  }
  return run_rounds_bytes_ws(k, decrypt, in, out, ks, T, k->d_gm, k->d_scratch, st, true);
}

// The byte kernels (any geometry): r launches over T frames, alternating
// between `out` and `scratch` (T frames) so that the last round lands in `out`.
cv_status run_rounds_bytes_ws(cv_key* k, bool decrypt, const uint8_t* in, uint8_t* out,
                              const uint8_t* ks, uint32_t T, const uint32_t* gm, uint8_t* scratch,
                              hipStream_t st, bool timed) {
  const uint32_t r = k->g.r;
  cv::RoundArgs a = round_args(k, ks, T);
  a.gm = gm;
  const uint8_t* cur = in;
  for (uint32_t s = 0; s < r; s++) {
    uint8_t* target = ((r - 1 - s) % 2 == 0) ? out : scratch;
    a.src = cur;
    a.dst = target;
    Timed tm(timed ? k : nullptr, st);
    if (!decrypt) {
      a.j = s;
      a.tile_rows = k->tile_enc;
      CV_HIP(cv::launch_round_enc(a, k->threads, st));
    } else {
      a.j = r - 1 - s;
      a.tile_rows = k->tile_dec;
      CV_HIP(cv::launch_round_dec(a, k->threads, st));
    }
    tm.end(1, T);
    cur = target;
  }
  return CV_OK;
}

cv_status check_frames_args(const cv_key* k, const uint8_t* in, uint8_t* out, const uint32_t* s_c,
                            size_t n) {
  if (!k) return fail(CV_E_INVAL, "key is NULL");
  if (n == 0) return CV_OK;
  if (!in || !out || !s_c) return fail(CV_E_INVAL, "NULL buffer");
  if (ranges_overlap(in, n * k->F, out, n * k->F)) return fail(CV_E_INVAL, "in and out overlap");
  for (size_t t = 0; t < n; t++)
    if (s_c[t] == 0) return fail(CV_E_INVAL, "confusion seed s_c must be >= 1");
  if (n > 0xFFFFFFFFull) return fail(CV_E_INVAL, "too many frames in one call");
  return CV_OK;
}

// One batch of T frames through a graph of its work (cv_launch.use_graph):
// the shift tables are written to the pinned staging buffer the graph copies
// from, then the graph captured for this buffer set is replayed (captured on
// the key's private stream the first time).  Everything else a capture
// records -- workspace, launch shape, chain descriptors -- is fixed until
// drop_graphs; what varies from call to call is in the signature.
cv_status crypt_batch_graph(cv_key* k, bool decrypt, const uint8_t* in, uint8_t* out,
                            const uint32_t* s_c, uint32_t T, hipStream_t st) {
  const Geom& g = k->g;
  if (k->gm_pending) {
    CV_HIP(hipEventSynchronize(k->gm_done));
    k->gm_pending = false;
  }
  for (uint32_t t = 0; t < T; t++) shift_table(g.H, g.W, s_c[t], k->h_gm + (uint64_t)t * g.H);
  const uint64_t sig[8] = {(uint64_t)decrypt, (uint64_t)(uintptr_t)in, (uint64_t)(uintptr_t)out, T,
                           (uint64_t)k->path, (uint64_t)prbg_variant(k), k->spin_limit, 0};
  cv_key::GraphEntry* e = nullptr;
  for (auto& x : k->graphs)
    if (memcmp(x.sig, sig, sizeof(sig)) == 0) e = &x;
  if (e) {
    k->graph_replays++;
  } else {
    if (!k->cap) CV_HIP(hipStreamCreateWithFlags(&k->cap, hipStreamNonBlocking));
    // the fused workspace (allocations are not allowed inside a capture)
    if (use_pw(k, in, out, k->d_ks) && k->path == CV_PATH_FUSED && k->fused_groups > 0) {
      cv_status s = ensure_fused(k);
      if (s == CV_OK && decrypt) s = ensure_rows_tables(k, T);
      if (s != CV_OK) return s;
    }
    if (k->graphs.size() >= cv_key::kMaxGraphs) {
      size_t lru = 0;
      for (size_t i = 1; i < k->graphs.size(); i++)
        if (k->graphs[i].last_use < k->graphs[lru].last_use) lru = i;
      CV_HIP(hipDeviceSynchronize());  // it may still be running
      (void)hipGraphExecDestroy(k->graphs[lru].exec);
      k->graphs.erase(k->graphs.begin() + lru);
    }
    CV_HIP(hipStreamBeginCapture(k->cap, hipStreamCaptureModeThreadLocal));
    k->capturing = true;
    k->captured_err = false;
    cv_status s = CV_OK;
    const hipError_t ce = hipMemcpyAsync(k->d_gm, k->h_gm, (uint64_t)T * g.H * sizeof(uint32_t),
                                         hipMemcpyHostToDevice, k->cap);
    if (ce != hipSuccess) s = hip_fail(ce, "hipMemcpyAsync (shift tables)");
    if (s == CV_OK) s = launch_keystream(k, k->d_ks, T, k->cap);
    if (s == CV_OK) s = run_rounds(k, decrypt, in, out, k->d_ks, T, k->cap);
    k->capturing = false;
    hipGraph_t graph = nullptr;
    const hipError_t ee = hipStreamEndCapture(k->cap, &graph);
    if (s != CV_OK || ee != hipSuccess) {
      if (graph) (void)hipGraphDestroy(graph);
      return s != CV_OK ? s : hip_fail(ee, "hipStreamEndCapture");
    }
    cv_key::GraphEntry ne{};
    memcpy(ne.sig, sig, sizeof(sig));
    ne.reads_err = k->captured_err;
    const hipError_t ie = hipGraphInstantiate(&ne.exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ie != hipSuccess) return hip_fail(ie, "hipGraphInstantiate");
    k->graphs.push_back(ne);
    e = &k->graphs.back();
    k->graph_captures++;
  }
  e->last_use = ++k->graph_clock;
  CV_HIP(hipGraphLaunch(e->exec, st));
  CV_HIP(hipEventRecord(k->gm_done, st));
  k->gm_pending = true;
  if (e->reads_err) {
    CV_HIP(hipEventRecord(k->err_copied, st));
    k->err_pending = true;
  }
  return CV_OK;
}

// ------------------------------------------------ keystream lookahead ---
hipError_t copy_sync(void* dst, const void* src, size_t bytes, hipMemcpyKind kind);

size_t state_doubles(const cv_key* k);

// Stream, events, shadow states and the chain tables that point at them.
cv_status side_stream(SideStreams& ss, int device, hipStream_t st, hipStream_t* out) {
  const bool null_stream = st == nullptr || st == hipStreamLegacy;
  hipStream_t& s = null_stream ? ss.plain : ss.own;
  if (!s) {
    hipError_t e = hipErrorNotSupported;
    if (!null_stream) {
      int cus = 0;
      e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device);
      std::vector<uint32_t> mask((std::max(cus, 1) + 31) / 32, 0xFFFFFFFFu);
      if (cus % 32) mask.back() = (1u << (cus % 32)) - 1;
      if (e == hipSuccess) e = hipExtStreamCreateWithCUMask(&s, (uint32_t)mask.size(), mask.data());
    }
    if (e != hipSuccess) {  // beside the null stream, or masks not supported
      (void)hipGetLastError();
      s = nullptr;
      CV_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    }
  }
  ss.last = s;
  *out = s;
  return CV_OK;
}

void side_streams_free(SideStreams& ss) {
  if (ss.plain) (void)hipStreamDestroy(ss.plain);
  if (ss.own) (void)hipStreamDestroy(ss.own);
  ss = SideStreams{};
}

cv_status ensure_ahead(cv_key* k) {
  cv_key::Ahead& a = k->ahead;
  if (a.ready) return CV_OK;
  // (after a failure, a later call completes what is missing)
  hipError_t e = hipSuccess;
  for (hipEvent_t* ev : {&a.ks_ready, &a.done[0], &a.done[1]})
    if (e == hipSuccess && !*ev) e = hipEventCreateWithFlags(ev, hipEventDisableTiming);
  const size_t nd = state_doubles(k);
  for (int i = 0; i < 2 && e == hipSuccess; i++) {
    if (!a.d_shadow[i]) e = hipMalloc(&a.d_shadow[i], nd * sizeof(double));
    if (e != hipSuccess) break;
    if (k->map == CV_MAP_2DLASM) {
      std::vector<cv::LasmChain> ch = k->h_lchains;
      for (cv::LasmChain& c : ch) c.state = a.d_shadow[i] + (c.state - k->d_state);
      if (!a.d_lchains[i]) e = hipMalloc(&a.d_lchains[i], ch.size() * sizeof(cv::LasmChain));
      if (e == hipSuccess)
        e = copy_sync(a.d_lchains[i], ch.data(), ch.size() * sizeof(cv::LasmChain),
                      hipMemcpyHostToDevice);
    } else {
      std::vector<cv::PlcmChain> ch = k->h_chains;
      for (cv::PlcmChain& c : ch) c.state = a.d_shadow[i] + (c.state - k->d_state);
      if (!a.d_chains[i]) e = hipMalloc(&a.d_chains[i], ch.size() * sizeof(cv::PlcmChain));
      if (e == hipSuccess)
        e = copy_sync(a.d_chains[i], ch.data(), ch.size() * sizeof(cv::PlcmChain),
                      hipMemcpyHostToDevice);
    }
  }
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(e == hipErrorOutOfMemory ? CV_E_NOMEM : CV_E_HIP, "lookahead set-up failed");
  }
  a.ready = true;
  return CV_OK;
}

// Keystream buffer i of at least `bytes`; a lookahead that wrote the old one is lost.
cv_status ahead_buffer(cv_key* k, int i, size_t bytes) {
  cv_key::Ahead& a = k->ahead;
  if (a.ks_cap[i] >= bytes) return CV_OK;
  CV_HIP(hipDeviceSynchronize());  // the old buffer may still be in use
  if (a.d_ks[i]) (void)hipFree(a.d_ks[i]);
  a.d_ks[i] = nullptr;
  a.ks_cap[i] = 0;
  if (a.target == i) a.valid = false;
  if (hipMalloc(&a.d_ks[i], bytes) != hipSuccess) {
    (void)hipGetLastError();
    a.d_ks[i] = nullptr;
    return fail(CV_E_NOMEM, "lookahead keystream allocation failed");
  }
  a.ks_cap[i] = bytes;
  return CV_OK;
}

// One internal batch of T frames with the lookahead: the keystream taken
// from the last lookahead when it predicted this batch (its shadow states
// become the key's), else generated on st; then the shadow copy for the next
// batch is made on st, the rounds run on st, and the next batch's keystream
// is generated on the private stream into the other buffer.
cv_status crypt_batch_ahead(cv_key* k, bool decrypt, const uint8_t* in, uint8_t* out,
                            const uint32_t* s_c, uint32_t T, hipStream_t st) {
  cv_key::Ahead& a = k->ahead;
  cv_status s = ensure_ahead(k);
  if (s != CV_OK) return s;
  const bool hit = a.valid && a.frame_index == k->frame_index && a.T == T && a.epoch == k->state_epoch;
  if (a.valid) (hit ? k->ahead_hits : k->ahead_misses)++;
  a.valid = false;
  const int buf = hit ? a.target : (a.target == 0 ? 1 : 0), nsh = a.shadow == 0 ? 1 : 0;
  const size_t bytes = (size_t)T * k->g.r * k->F, states = state_doubles(k) * sizeof(double);
  if ((s = ahead_buffer(k, buf, bytes)) != CV_OK) return s;
  if ((s = ahead_buffer(k, 1 - buf, bytes)) != CV_OK) return s;
  if ((s = upload_shift_tables(k, s_c, T, st)) != CV_OK) return s;
  if (hit) {
    CV_HIP(hipStreamWaitEvent(st, a.done[a.shadow], 0));
    CV_HIP(hipMemcpyAsync(k->d_state, a.d_shadow[a.shadow], states, hipMemcpyDeviceToDevice, st));
    // a 2DLASM lookahead's undecided sine (the key's error word) is read back here
    if (k->map == CV_MAP_2DLASM && (s = queue_err_readback(k, st)) != CV_OK) return s;
  } else if ((s = launch_keystream(k, a.d_ks[buf], T, st)) != CV_OK) {
    return s;
  }
  if (a.used[nsh]) CV_HIP(hipStreamWaitEvent(st, a.done[nsh], 0));
  CV_HIP(hipMemcpyAsync(a.d_shadow[nsh], k->d_state, states, hipMemcpyDeviceToDevice, st));
  CV_HIP(hipEventRecord(a.ks_ready, st));
  if ((s = run_rounds(k, decrypt, in, out, a.d_ks[buf], T, st)) != CV_OK) return s;
  k->frame_index += T;
  hipStream_t ps = nullptr;
  if ((s = side_stream(a.side, k->device, st, &ps)) != CV_OK) return s;
  CV_HIP(hipStreamWaitEvent(ps, a.ks_ready, 0));
  {
    Timed tm(k, ps);
    if (k->map == CV_MAP_2DLASM)
      CV_HIP(cv::launch_prbg_lasm(a.d_lchains[nsh], k->g.n, a.d_ks[1 - buf], T, 0, k->d_err, ps));
    else
      CV_HIP(cv::launch_prbg_plcm(a.d_chains[nsh], k->g.n, a.d_ks[1 - buf], T, prbg_variant(k), ps));
    tm.end(0, prbg_steps(k, T));
  }
  CV_HIP(hipEventRecord(a.done[nsh], ps));
  a.used[nsh] = true;
  a.target = 1 - buf;
  a.shadow = nsh;
  a.frame_index = k->frame_index;
  a.epoch = k->state_epoch;
  a.T = T;
  a.valid = true;
  return CV_OK;
}

// A stream that a caller is capturing into a graph of its own is left alone:
// the captured work runs when the caller launches the graph, which the
// caller orders.
bool capturing(hipStream_t st) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(st, &cs) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return cs != hipStreamCaptureStatusNone;
}

cv_status key_order_wait(const cv_key* k, hipStream_t st) {
  if (k->order_has && k->order_stream != st && !capturing(st))
    CV_HIP(hipStreamWaitEvent(st, k->order_ev, 0));
  return CV_OK;
}

cv_status key_order_mark(cv_key* k, hipStream_t st) {
  if (capturing(st)) {
    k->order_has = false;
    return CV_OK;
  }
  if (!k->order_ev) CV_HIP(hipEventCreateWithFlags(&k->order_ev, hipEventDisableTiming));
  CV_HIP(hipEventRecord(k->order_ev, st));
  k->order_stream = st;
  k->order_has = true;
  return CV_OK;
}

// The end of a call that took stream st: mark the key's order there, also
// behind the work a failed call enqueued (keeping the call's own error).
cv_status key_order_done(cv_key* k, hipStream_t st, cv_status s) {
  if (s == CV_OK) return key_order_mark(k, st);
  const std::string msg = g_last_error;
  (void)key_order_mark(k, st);
  return fail(s, msg);
}

cv_status crypt_frames_ordered(cv_key* k, bool decrypt, const uint8_t* in, uint8_t* out,
                               const uint32_t* s_c, size_t n, hipStream_t st);

cv_status crypt_frames(cv_key* k, bool decrypt, const uint8_t* in, uint8_t* out,
                       const uint32_t* s_c, size_t n, void* stream) {
  cv_status s = check_frames_args(k, in, out, s_c, n);
  if (s != CV_OK || n == 0) return s;
  if ((s = check_async_errors(k, false)) != CV_OK) return s;
  DeviceGuard dg(k->device);
  hipStream_t st = (hipStream_t)stream;
  if ((s = key_order_wait(k, st)) != CV_OK) return s;
  return key_order_done(k, st, crypt_frames_ordered(k, decrypt, in, out, s_c, n, st));
}

cv_status crypt_frames_ordered(cv_key* k, bool decrypt, const uint8_t* in, uint8_t* out,
                               const uint32_t* s_c, size_t n, hipStream_t st) {
  cv_status s = CV_OK;
  const size_t B = std::min<size_t>(n, k->batch_frames);
  if ((s = ensure_workspace(k, B)) != CV_OK) return s;
  const bool ahead = k->lookahead;
  const bool graph = k->use_graph && !k->profiling && !ahead;
  for (size_t f0 = 0; f0 < n; f0 += B) {
    const uint32_t T = (uint32_t)std::min(B, n - f0);
    if (ahead) {
      if ((s = crypt_batch_ahead(k, decrypt, in + f0 * k->F, out + f0 * k->F, s_c + f0, T, st)) !=
          CV_OK)
        return s;
      continue;  // the batch advanced frame_index
    }
    if (graph) {
      if ((s = crypt_batch_graph(k, decrypt, in + f0 * k->F, out + f0 * k->F, s_c + f0, T, st)) !=
          CV_OK)
        return s;
    } else {
      if ((s = upload_shift_tables(k, s_c + f0, T, st)) != CV_OK) return s;
      if ((s = launch_keystream(k, k->d_ks, T, st)) != CV_OK) return s;
      if ((s = run_rounds(k, decrypt, in + f0 * k->F, out + f0 * k->F, k->d_ks, T, st)) != CV_OK)
        return s;
    }
    k->frame_index += T;
  }
  return CV_OK;
}

bool finite_in(double v, double lo, double hi) { return isfinite(v) && v > lo && v < hi; }

size_t state_doubles(const cv_key* k) { return (k->map == CV_MAP_2DLASM ? 4ull : 2ull) * k->g.n; }

// Sec. 3, Eq. (6): the control parameter's admissible set.
bool lasm_mu_ok(double mu) {
  return (mu >= 0.37 && mu <= 0.38) || (mu >= 0.4 && mu <= 0.42) || (mu >= 0.44 && mu <= 0.93) ||
         mu == 1.0;
}

cv_status ensure_err_flag(cv_key* k);
hipError_t copy_sync(void* dst, const void* src, size_t bytes, hipMemcpyKind kind);

// Generators of a 2DLASM key: per band two maps (x0, y0, mu) of Eq. (6).
cv_status setup_lasm(cv_key* k, const double* p_m) {
  const Geom& g = k->g;
  const uint64_t row = (uint64_t)g.W * g.C;
  std::vector<double> state(4 * g.n);
  std::vector<cv::LasmChain> chains(g.n);
  if (hipMalloc(&k->d_state, state.size() * sizeof(double)) != hipSuccess ||
      hipMalloc(&k->d_lchains, chains.size() * sizeof(cv::LasmChain)) != hipSuccess) {
    (void)hipGetLastError();
    return fail(CV_E_NOMEM, "key allocation failed");
  }
  k->fast = false;
  for (uint32_t i = 0; i < g.n; i++) {
    const double* q = p_m + 6 * i;
    cv::LasmChain& c = chains[i];
    c.state = k->d_state + 4 * i;
    for (int m = 0; m < 2; m++) {
      state[4 * i + 2 * m] = q[3 * m];
      state[4 * i + 2 * m + 1] = q[3 * m + 1];
      c.mu[m] = q[3 * m + 2];
    }
    const uint64_t lo = cv::band_lo(g.H, g.n, i), hi = cv::band_lo(g.H, g.n, i + 1);
    c.out_off = (uint64_t)g.r * lo * row;
    c.frame_stride = (uint64_t)g.r * k->F;
    c.nbytes = (uint64_t)g.r * (hi - lo) * row;
  }
  hipError_t e = copy_sync(k->d_state, state.data(), state.size() * sizeof(double),
                           hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = copy_sync(k->d_lchains, chains.data(), chains.size() * sizeof(cv::LasmChain),
                  hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&k->gm_done, hipEventDisableTiming);
  if (e != hipSuccess) return hip_fail(e, "cv_keysetup");
  k->h_lchains = chains;
  return ensure_err_flag(k);
}

// Blocking host<->device copy on a private non-blocking stream of the current
// device, so that it waits for no other stream (the legacy null stream would
// wait for every blocking stream, compute-unit-masked ones included).
hipError_t copy_sync(void* dst, const void* src, size_t bytes, hipMemcpyKind kind) {
  static std::mutex mu;
  static std::vector<hipStream_t> streams;  // per device
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  hipStream_t st = nullptr;
  {
    std::lock_guard<std::mutex> g(mu);
    if ((int)streams.size() <= dev) streams.resize(dev + 1, nullptr);
    if (!streams[dev] && (e = hipStreamCreateWithFlags(&streams[dev], hipStreamNonBlocking)) != hipSuccess)
      return e;
    st = streams[dev];
  }
  e = hipMemcpyAsync(dst, src, bytes, kind, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  return e;
}

}  // namespace rt
}  // namespace cv

using namespace cv::rt;

extern "C" {

int cv_spec_version(void) { return CV_SPEC_VERSION; }

const char* cv_last_error(void) { return g_last_error.c_str(); }

cv_status cv_keysetup(const cv_geom* geom, cv_map map, const double* p_m, size_t n_doubles,
                      int device, cv_key** out) {
  if (!geom || !p_m || !out) return fail(CV_E_INVAL, "NULL argument");
  *out = nullptr;
  const Geom g{geom->height, geom->width, geom->channels, geom->n_sub, geom->rounds};
  if (map != CV_MAP_PLCM && map != CV_MAP_2DLASM) return fail(CV_E_INVAL, "unknown map");
  const uint32_t rec = map == CV_MAP_PLCM ? 4 : 6;  // doubles per subframe record
  if (!g.H || !g.W || !g.C || !g.n || !g.r) return fail(CV_E_INVAL, "zero in geometry");
  if (g.n > g.H) return fail(CV_E_INVAL, "more subframes than rows");
  const uint64_t row = (uint64_t)g.W * g.C;
  if ((uint64_t)g.H * row > 0xFFFFFFFFull / 8) return fail(CV_E_INVAL, "frame too large");
  if (n_doubles != (uint64_t)rec * g.n)
    return fail(CV_E_INVAL, map == CV_MAP_PLCM ? "p_m must hold 4 doubles per subframe"
                                               : "p_m must hold 6 doubles per subframe");
  for (uint32_t i = 0; i < g.n; i++) {
    const uint64_t S = (cv::band_lo(g.H, g.n, i + 1) - cv::band_lo(g.H, g.n, i)) * row;
    if (S < 2) return fail(CV_E_INVAL, "every subframe needs at least 2 bytes");
    const double* q = p_m + (uint64_t)rec * i;
    if (map == CV_MAP_PLCM) {
      if (!finite_in(q[0], 0.0, 1.0) || !finite_in(q[2], 0.0, 1.0))
        return fail(CV_E_INVAL, "PLCM x0 must lie in (0,1)");
      if (!finite_in(q[1], 0.0, 0.5) || !finite_in(q[3], 0.0, 0.5))
        return fail(CV_E_INVAL, "PLCM p must lie in (0,1/2)");
    } else {
      for (int m = 0; m < 2; m++) {
        if (!finite_in(q[3 * m], 0.0, 1.0) || !finite_in(q[3 * m + 1], 0.0, 1.0))
          return fail(CV_E_INVAL, "2DLASM x0 and y0 must lie in (0,1)");
        if (!lasm_mu_ok(q[3 * m + 2]))
          return fail(CV_E_INVAL, "2DLASM mu must lie in [0.37,0.38], [0.4,0.42], [0.44,0.93] or be 1");
      }
      // one launch covers a batch of frames: a chain's steps must fit 31 bits
      if ((uint64_t)g.r * S > (1ull << 31)) return fail(CV_E_INVAL, "subframe too large");
    }
  }
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
    return fail(CV_E_INVAL, "no such HIP device");
  DeviceGuard dg(device);
  const size_t lds_max = lds_limit(device);
  if (cv::round_lds_bytes(g, 1) > lds_max) return fail(CV_E_INVAL, "row too wide for LDS");

  static std::atomic<uint64_t> serials{0};
  cv_key* k = new cv_key();
  k->serial = ++serials;
  k->g = g;
  k->map = map;
  k->device = device;
  k->F = (uint64_t)g.H * row;
  k->pm.assign(p_m, p_m + n_doubles);
  // launch shape: LDS tiles of up to 64 KiB (two workgroups per CU)
  const size_t budget = std::min<size_t>(lds_max, 64 * 1024);
  uint32_t rows_fit = 1;
  while (rows_fit < g.H && cv::round_lds_bytes(g, rows_fit + 1) <= budget) rows_fit++;
  uint32_t max_band_rows = 0;
  for (uint32_t i = 0; i < g.n; i++)
    max_band_rows = std::max<uint32_t>(
        max_band_rows, (uint32_t)(cv::band_lo(g.H, g.n, i + 1) - cv::band_lo(g.H, g.n, i)));
  k->max_band_rows = max_band_rows;
  k->lds_max = lds_max;
  k->tile_enc = std::min({rows_fit, max_band_rows, k->threads});
  k->tile_dec = std::min({rows_fit, g.H, k->threads});
  k->tile_pw = pw_tile_rows(g, k->threads, lds_max);
  set_fused_groups(k, 0);
  // batches of frames: keystream + scratch within ~1 GiB
  const uint64_t per_frame = (uint64_t)(g.r + 1) * k->F;
  k->batch_frames = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(256, (1ull << 30) / per_frame));

  if (map == CV_MAP_2DLASM) {
    cv_status st = setup_lasm(k, p_m);
    if (st != CV_OK) {
      cv_key_free(k);
      return st;
    }
    *out = k;
    return CV_OK;
  }
  std::vector<double> state(2 * g.n);
  std::vector<cv::PlcmChain> chains(g.n);
  if (hipMalloc(&k->d_state, state.size() * sizeof(double)) != hipSuccess ||
      hipMalloc(&k->d_chains, chains.size() * sizeof(cv::PlcmChain)) != hipSuccess) {
    (void)hipGetLastError();
    cv_key_free(k);
    return fail(CV_E_NOMEM, "key allocation failed");
  }
  k->fast = true;
  for (uint32_t i = 0; i < g.n; i++) {
    const double* q = p_m + 4 * i;
    state[2 * i] = q[0];
    state[2 * i + 1] = q[2];
    cv::PlcmChain& c = chains[i];
    c.state = k->d_state + 2 * i;
    for (int m = 0; m < 2; m++) {
      c.p[m] = q[2 * m + 1];
      c.h[m] = 0.5 - c.p[m];
      c.ip[m] = 1.0 / c.p[m];
      c.ih[m] = 1.0 / c.h[m];
      // 1 - RN(1/d)*d is exact (one FMA), so dividing it by d gives RN(1/d - RN(1/d))
      c.lp[m] = std::fma(-c.ip[m], c.p[m], 1.0) / c.p[m];
      c.lh[m] = std::fma(-c.ih[m], c.h[m], 1.0) / c.h[m];
      k->fast = k->fast && cv::plcm_fast_ok(q[2 * m], c.p[m]);
    }
    const uint64_t lo = cv::band_lo(g.H, g.n, i), hi = cv::band_lo(g.H, g.n, i + 1);
    c.out_off = (uint64_t)g.r * lo * row;
    c.frame_stride = (uint64_t)g.r * k->F;
    c.nbytes = (uint64_t)g.r * (hi - lo) * row;
  }
  hipError_t e = copy_sync(k->d_state, state.data(), state.size() * sizeof(double),
                           hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = copy_sync(k->d_chains, chains.data(), chains.size() * sizeof(cv::PlcmChain),
                  hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&k->gm_done, hipEventDisableTiming);
  k->h_chains = chains;
  if (e != hipSuccess) {
    cv_key_free(k);
    return hip_fail(e, "cv_keysetup");
  }
  *out = k;
  return CV_OK;
}

void cv_key_free(cv_key* k) {
  if (!k) return;
  DeviceGuard dg(k->device);
  (void)hipDeviceSynchronize();
  (void)drain_spans(k);
  for (hipEvent_t e : k->event_pool) (void)hipEventDestroy(e);
  free_workspace(k);
  if (k->cap) (void)hipStreamDestroy(k->cap);
  if (k->d_fscratch) (void)hipFree(k->d_fscratch);
  if (k->d_counters) (void)hipFree(k->d_counters);
  if (k->d_rows_tables) (void)hipFree(k->d_rows_tables);
  if (k->order_ev) (void)hipEventDestroy(k->order_ev);
  if (k->d_err) (void)hipFree(k->d_err);
  if (k->h_err) (void)hipHostFree(k->h_err);
  if (k->err_copied) (void)hipEventDestroy(k->err_copied);
  if (k->d_state) (void)hipFree(k->d_state);
  if (k->d_chains) (void)hipFree(k->d_chains);
  if (k->d_lchains) (void)hipFree(k->d_lchains);
  if (k->gm_done) (void)hipEventDestroy(k->gm_done);
  cv_key::Ahead& a = k->ahead;
  for (int i = 0; i < 2; i++) {
    if (a.d_shadow[i]) (void)hipFree(a.d_shadow[i]);
    if (a.d_chains[i]) (void)hipFree(a.d_chains[i]);
    if (a.d_lchains[i]) (void)hipFree(a.d_lchains[i]);
    if (a.d_ks[i]) (void)hipFree(a.d_ks[i]);
    if (a.done[i]) (void)hipEventDestroy(a.done[i]);
  }
  if (a.ks_ready) (void)hipEventDestroy(a.ks_ready);
  side_streams_free(a.side);
  delete k;
}

cv_status cv_key_get_state(const cv_key* k, double* x, size_t n_doubles, uint64_t* frame_index) {
  if (!k || !x || !frame_index) return fail(CV_E_INVAL, "NULL argument");
  if (n_doubles != state_doubles(k))
    return fail(CV_E_INVAL, "state holds 2 (PLCM) or 4 (2DLASM) doubles per subframe");
  DeviceGuard dg(k->device);
  CV_HIP(hipDeviceSynchronize());
  cv_status s = check_async_errors(const_cast<cv_key*>(k), true);
  if (s != CV_OK) return s;
  CV_HIP(hipMemcpy(x, k->d_state, n_doubles * sizeof(double), hipMemcpyDeviceToHost));
  *frame_index = k->frame_index;
  return CV_OK;
}

cv_status cv_key_set_state(cv_key* k, const double* x, size_t n_doubles, uint64_t frame_index) {
  if (!k || !x) return fail(CV_E_INVAL, "NULL argument");
  if (n_doubles != state_doubles(k))
    return fail(CV_E_INVAL, "state holds 2 (PLCM) or 4 (2DLASM) doubles per subframe");
  for (size_t i = 0; i < n_doubles; i++)
    if (!(x[i] >= 0.0 && x[i] <= 1.0)) return fail(CV_E_INVAL, "state outside [0,1]");
  DeviceGuard dg(k->device);
  CV_HIP(hipDeviceSynchronize());
  cv_status s = check_async_errors(k, true);
  if (s != CV_OK) return s;
  CV_HIP(hipMemcpy(k->d_state, x, n_doubles * sizeof(double), hipMemcpyHostToDevice));
  k->frame_index = frame_index;
  k->state_epoch++;
  if (k->map == CV_MAP_PLCM) {
    bool fast = true;
    for (uint32_t i = 0; i < k->g.n; i++)
      for (int m = 0; m < 2; m++) fast = fast && cv::plcm_fast_ok(x[2 * i + m], k->pm[4 * i + 2 * m + 1]);
    k->fast = fast;
  }
  return CV_OK;
}

cv_status cv_key_set_path(cv_key* k, int path) {
  if (!k) return fail(CV_E_INVAL, "key is NULL");
  if (path != CV_PATH_PLAIN && path != CV_PATH_FUSED) return fail(CV_E_INVAL, "unknown path");
  k->path = path;
  return CV_OK;
}

cv_status cv_key_sync(cv_key* k) {
  if (!k) return fail(CV_E_INVAL, "key is NULL");
  DeviceGuard dg(k->device);
  CV_HIP(hipDeviceSynchronize());
  return check_async_errors(k, true);
}

cv_status cv_key_set_spin_limit(cv_key* k, uint32_t polls) {
  if (!k) return fail(CV_E_INVAL, "key is NULL");
  k->spin_limit = polls;
  return CV_OK;
}

cv_status cv_key_get_launch(const cv_key* k, cv_launch* l) {
  if (!k || !l) return fail(CV_E_INVAL, "NULL argument");
  l->batch_frames = k->batch_frames;
  l->threads = k->threads;
  l->tile_rows_enc = k->tile_enc;
  l->tile_rows_dec = k->tile_dec;
  l->prbg_variant = k->prbg_variant;
  l->round_variant = k->round_variant;
  l->tile_rows_pw = k->tile_pw;
  l->fused_groups = k->fused_groups;
  l->use_graph = k->use_graph ? 1u : 0u;
  l->lookahead = k->lookahead ? 1u : 0u;
  return CV_OK;
}

cv_status cv_key_autotune(cv_key* k, int decrypt, uint32_t n_frames, void* stream, cv_launch* best,
                          int* cached) {
  if (!k) return fail(CV_E_INVAL, "key is NULL");
  if (n_frames == 0) return fail(CV_E_INVAL, "n_frames must be >= 1");
  if (cached) *cached = 0;
  const Geom& g = k->g;
  if (!((g.C == 3 || g.C == 4) && g.W % 16 == 0) || k->tile_pw == 0)
    return fail(CV_E_INVAL, "the fused path needs C in {3,4} and W a multiple of 16");
  cv_status s = check_async_errors(k, false);
  if (s != CV_OK) return s;
  DeviceGuard dg(k->device);
  hipStream_t st = (hipStream_t)stream;
  char kb[160];
  snprintf(kb, sizeof kb, "key|lds%zu|%ux%ux%u/n%u/r%u/%c%u", k->lds_max, g.H, g.W, g.C, g.n, g.r,
           decrypt ? 'd' : 'e', n_frames);
  const std::string key = kb;
  cv_launch cur{};
  (void)cv_key_get_launch(k, &cur);
  cur.batch_frames = std::max(cur.batch_frames, n_frames);  // one batch per call
  std::map<std::string, int64_t> f;
  if (tune_lookup(key, &f) && f.count("round_variant") && f.count("threads") &&
      f.count("fused_groups")) {
    cv_launch l = cur;
    l.round_variant = (uint32_t)f["round_variant"];
    l.threads = (uint32_t)f["threads"];
    l.fused_groups = (uint32_t)f["fused_groups"];
    if (cv_key_set_launch(k, &l) == CV_OK) {
      k->path = CV_PATH_FUSED;
      if (cached) *cached = 1;
      if (best) (void)cv_key_get_launch(k, best);
      return CV_OK;
    }
  }
  // scratch frames and keystream (their bytes do not change the timing)
  const uint64_t F = k->F, bytes = (uint64_t)n_frames * F;
  uint8_t *d_in = nullptr, *d_out = nullptr, *d_ks = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  auto release = [&]() {
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (d_in) (void)hipFree(d_in);
    if (d_out) (void)hipFree(d_out);
    if (d_ks) (void)hipFree(d_ks);
  };
  if (hipMalloc(&d_in, bytes) != hipSuccess || hipMalloc(&d_out, bytes) != hipSuccess ||
      hipMalloc(&d_ks, bytes * g.r) != hipSuccess) {
    (void)hipGetLastError();
    release();
    return fail(CV_E_NOMEM, "autotuner scratch allocation failed");
  }
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    release();
    return hip_fail(hipErrorOutOfMemory, "hipEventCreate");
  }
  std::vector<uint32_t> seeds(n_frames);
  for (uint32_t t = 0; t < n_frames; t++) seeds[t] = 1 + t;
  const bool dec = decrypt != 0;
  cv_launch win = cur;
  float win_ms = -1.f;
  // candidates: the fused kernels (pixel-word with 512 or 1024 threads,
  // row-run) and the frame groups in flight, 8 at a time up to the capacity
  for (uint32_t variant : {2u, 3u}) {
    for (uint32_t th : {512u, 1024u}) {
      if (variant == 3 && th != 1024) continue;
      for (uint32_t groups = 8;; groups += 8) {
        cv_launch l = cur;
        l.round_variant = variant;
        l.threads = th;
        l.fused_groups = groups;
        if (cv_key_set_launch(k, &l) != CV_OK) break;
        if (fused_group_cap(k, dec) < groups) break;  // beyond the resident capacity
        if (variant == 3 && fused_kernel(k, dec) == FUSED_PW) break;  // no row-run kernel here
        if ((s = ensure_workspace(k, n_frames)) != CV_OK || (s = ensure_fused(k)) != CV_OK ||
            (dec && (s = ensure_rows_tables(k, n_frames)) != CV_OK) ||
            (s = upload_shift_tables(k, seeds.data(), n_frames, st)) != CV_OK)
          break;
        float ms = 0.f;
        for (int rep = 0; rep < 4 && s == CV_OK; rep++) {
          if (rep == 1 && hipEventRecord(e0, st) != hipSuccess) s = hip_fail(hipErrorUnknown, "hipEventRecord");
          if (s == CV_OK)
            s = launch_fused_ws(k, dec, d_in, d_out, d_ks, n_frames, k->d_gm, k->d_fscratch,
                                k->d_counters, k->d_err, k->fused_groups, st, k->d_rows_tables);
        }
        if (s != CV_OK) break;
        if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
          s = hip_fail(hipErrorUnknown, "autotuner timing");
          break;
        }
        ms /= 3.f;
        if (win_ms < 0 || ms < win_ms) {
          win_ms = ms;
          win = l;
        }
      }
      if (s != CV_OK) break;
    }
    if (s != CV_OK) break;
  }
  (void)hipStreamSynchronize(st);
  release();
  if (s != CV_OK) {
    (void)cv_key_set_launch(k, &cur);
    return s;
  }
  if ((s = check_async_errors(k, true)) != CV_OK) return s;
  if ((s = cv_key_set_launch(k, &win)) != CV_OK) return s;
  k->path = CV_PATH_FUSED;
  (void)tune_store(key, {{"round_variant", win.round_variant}, {"threads", win.threads},
                         {"fused_groups", k->fused_groups}});
  if (best) (void)cv_key_get_launch(k, best);
  return CV_OK;
}

cv_status cv_key_graph_counts(const cv_key* k, uint64_t* captures, uint64_t* replays) {
  if (!k || !captures || !replays) return fail(CV_E_INVAL, "NULL argument");
  *captures = k->graph_captures;
  *replays = k->graph_replays;
  return CV_OK;
}

cv_status cv_key_lookahead_counts(const cv_key* k, uint64_t* hits, uint64_t* misses) {
  if (!k || !hits || !misses) return fail(CV_E_INVAL, "NULL argument");
  *hits = k->ahead_hits;
  *misses = k->ahead_misses;
  return CV_OK;
}

cv_status cv_key_set_launch(cv_key* k, const cv_launch* l) {
  if (!k || !l) return fail(CV_E_INVAL, "NULL argument");
  if (l->batch_frames == 0) return fail(CV_E_INVAL, "batch_frames must be >= 1");
  if (l->prbg_variant > 5) return fail(CV_E_INVAL, "prbg_variant must be 0..5");
  if (l->round_variant > 3) return fail(CV_E_INVAL, "round_variant must be 0..3");
  if (l->use_graph > 1) return fail(CV_E_INVAL, "use_graph must be 0 or 1");
  if (l->lookahead > 1) return fail(CV_E_INVAL, "lookahead must be 0 or 1");
  const uint32_t tp = pw_tile_limit(k->g, l->threads, l->tile_rows_pw);
  if (tp == 0 && (k->g.C == 3 || k->g.C == 4))
    return fail(CV_E_INVAL, "tile_rows_pw must be >= 1 (and the frame not too wide for threads)");
  if (cv::round_pw_lds_bytes(k->g, tp) > k->lds_max)
    return fail(CV_E_INVAL, "pixel-word tile does not fit in LDS");
  if (l->threads < 64 || l->threads > 1024 || l->threads % 64)
    return fail(CV_E_INVAL, "threads must be a multiple of 64 in 64..1024");
  const uint32_t te = std::min(l->tile_rows_enc, k->max_band_rows);
  const uint32_t td = std::min(l->tile_rows_dec, k->g.H);
  if (te == 0 || td == 0) return fail(CV_E_INVAL, "tile rows must be >= 1");
  if (te > l->threads || td > l->threads) return fail(CV_E_INVAL, "tile rows exceed threads");
  if (cv::round_lds_bytes(k->g, std::max(te, td)) > k->lds_max)
    return fail(CV_E_INVAL, "tile does not fit in LDS");
  k->batch_frames = l->batch_frames;
  k->threads = l->threads;
  k->tile_enc = te;
  k->tile_dec = td;
  k->prbg_variant = l->prbg_variant;
  k->round_variant = l->round_variant;
  k->tile_pw = tp;
  k->use_graph = l->use_graph != 0;
  k->lookahead = l->lookahead != 0;
  drop_graphs(k);
  // the fused workspace depends on the shape: drop it and size it anew
  if (k->d_fscratch) {
    CV_HIP(hipDeviceSynchronize());
    (void)hipFree(k->d_fscratch);
    (void)hipFree(k->d_counters);
    k->d_fscratch = nullptr;
    k->d_counters = nullptr;
  }
  set_fused_groups(k, l->fused_groups);
  return CV_OK;
}

cv_status cv_key_set_profiling(cv_key* k, int on) {
  if (!k) return fail(CV_E_INVAL, "key is NULL");
  DeviceGuard dg(k->device);
  cv_status s = drain_spans(k);
  if (s != CV_OK) return s;
  k->profiling = on != 0;
  k->prof = cv_profile{};
  return CV_OK;
}

cv_status cv_key_get_profile(cv_key* k, cv_profile* prof) {
  if (!k || !prof) return fail(CV_E_INVAL, "NULL argument");
  if (!k->profiling) return fail(CV_E_STATE, "profiling is off");
  DeviceGuard dg(k->device);
  cv_status s = drain_spans(k);
  if (s != CV_OK) return s;
  *prof = k->prof;
  return CV_OK;
}

cv_status cv_encrypt_frames(cv_key* k, const uint8_t* in, uint8_t* out, const uint32_t* s_c,
                            size_t n, void* stream) {
  return crypt_frames(k, false, in, out, s_c, n, stream);
}

cv_status cv_decrypt_frames(cv_key* k, const uint8_t* in, uint8_t* out, const uint32_t* s_c,
                            size_t n, void* stream) {
  return crypt_frames(k, true, in, out, s_c, n, stream);
}

cv_status cv_cr_sin(const double* t, double* out, size_t n, int force_exact, uint32_t* undecided,
                    void* stream) {
  if (n == 0) return CV_OK;
  if (!t || !out || !undecided) return fail(CV_E_INVAL, "NULL argument");
  CV_HIP(cv::launch_cr_sin(t, out, n, force_exact != 0, undecided, (hipStream_t)stream));
  return CV_OK;
}

cv_status cv_keystream_frames(cv_key* k, uint8_t* ks, size_t n, void* stream) {
  if (!k) return fail(CV_E_INVAL, "key is NULL");
  if (n == 0) return CV_OK;
  if (!ks) return fail(CV_E_INVAL, "NULL buffer");
  if (n > 0xFFFFFFFFull) return fail(CV_E_INVAL, "too many frames in one call");
  cv_status s = check_async_errors(k, false);
  if (s != CV_OK) return s;
  DeviceGuard dg(k->device);
  hipStream_t st = (hipStream_t)stream;
  if ((s = key_order_wait(k, st)) != CV_OK) return s;
  if ((s = launch_keystream(k, ks, (uint32_t)n, st)) == CV_OK) k->frame_index += n;
  return key_order_done(k, st, s);
}

cv_status cv_apply_rounds(cv_key* k, int decrypt, const uint8_t* in, uint8_t* out,
                          const uint8_t* ks, const uint32_t* s_c, size_t n, void* stream) {
  cv_status s = check_frames_args(k, in, out, s_c, n);
  if (s != CV_OK || n == 0) return s;
  if (!ks) return fail(CV_E_INVAL, "NULL keystream");
  if ((s = check_async_errors(k, false)) != CV_OK) return s;
  const size_t ks_bytes = n * (uint64_t)k->g.r * k->F;
  if (ranges_overlap(ks, ks_bytes, in, n * k->F) || ranges_overlap(ks, ks_bytes, out, n * k->F))
    return fail(CV_E_INVAL, "keystream overlaps a frame buffer");
  DeviceGuard dg(k->device);
  hipStream_t st = (hipStream_t)stream;
  const size_t B = std::min<size_t>(n, k->batch_frames);
  if ((s = ensure_workspace(k, B)) != CV_OK) return s;
  if ((s = key_order_wait(k, st)) != CV_OK) return s;
  for (size_t f0 = 0; f0 < n && s == CV_OK; f0 += B) {
    const uint32_t T = (uint32_t)std::min(B, n - f0);
    if ((s = upload_shift_tables(k, s_c + f0, T, st)) == CV_OK)
      s = run_rounds(k, decrypt != 0, in + f0 * k->F, out + f0 * k->F,
                     ks + f0 * (uint64_t)k->g.r * k->F, T, st);
  }
  return key_order_done(k, st, s);
}

}  // extern "C"
