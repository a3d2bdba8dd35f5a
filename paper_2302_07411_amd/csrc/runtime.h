// Host-side runtime state of libchaosvid shared by the C-ABI translation
// units (abi.cpp: keys; batch_host.cpp: multi-stream batches).
#pragma once
#include <map>
#include <string>
#include <vector>

#include "chaosvid.h"
#include "cv_internal.h"

using cv::Geom;

// Private streams for work that runs beside a caller's stream st (a key's
// lookahead, a batch's prefetch), chosen per call.  Beside the legacy null
// stream: a non-blocking stream, so that null-stream work does not wait for
// the private work.  Beside any other stream: a stream with a compute-unit
// mask of every CU, which gets a hardware queue of its own (a plain stream
// may share st's queue, and st's later work would then wait behind the
// private work); such a stream is ordered with the null stream, which st is
// not.  Consecutive private launches are ordered by the callers' events, not
// by the stream.
struct SideStreams {
  hipStream_t plain = nullptr;  // non-blocking
  hipStream_t own = nullptr;    // masked (or plain where masks are not supported)
  hipStream_t last = nullptr;   // the stream of the last private work
};

// One video stream's key: device-resident generator state plus the
// workspace its calls reuse.
struct cv_key {
  Geom g{};
  cv_map map = CV_MAP_PLCM;
  int device = 0;
  int path = CV_PATH_PLAIN;
  uint64_t F = 0;              // bytes per frame
  uint64_t frame_index = 0;    // frames processed so far
  uint64_t serial = 0;         // unique per key in the process (never reused)
  uint64_t state_epoch = 0;    // bumped whenever the generator state is set from outside
  std::vector<double> pm;      // the n key records as given
  double* d_state = nullptr;   // 2n: x of map 1, map 2 per band
  bool fast = false;           // every chain qualifies for the reciprocal division
  uint32_t prbg_variant = 0;   // requested generator variant (cv_launch.prbg_variant)
  uint32_t round_variant = 0;  // requested round kernels (cv_launch.round_variant)
  uint32_t tile_pw = 0;        // rows per LDS tile of the pixel-word kernels
  uint8_t* d_scratch2 = nullptr;  // second pixel-word scratch buffer
  // fused path: per resident group two pixel-word frames, a barrier counter,
  // and a timeout flag copied back to pinned memory after every launch
  uint32_t fused_groups = 0;   // groups in flight (<= resident capacity)
  uint32_t fused_cap = 0;      // resident capacity for the current launch shape
  uint32_t tile_skew = 0;      // rows per LDS tile of the row-run encryption kernel (0 = n/a)
  uint32_t fused_cap_skew = 0; // its resident capacity in groups
  uint32_t fused_cap_unskew = 0;  // resident groups of the row-run decryption kernel (0 = n/a)
  // decryption where a band exceeds one LDS tile: the row-run batch kernel
  // over the key's frames, tile by tile (0 = n/a)
  uint32_t rows_tile_dec = 0;  // its LDS tile rows
  uint32_t rows_G = 0;         // workgroups per group
  uint32_t rows_KQ = 0;        // kernel instance (the run width of its encryption code)
  size_t rows_lds = 0;
  uint32_t fused_cap_rows = 0; // its resident capacity in groups
  uint8_t* d_rows_tables = nullptr;  // its device-written job and slot tables
  size_t rows_tables_cap = 0;
  uint8_t* d_fscratch = nullptr;
  uint32_t* d_counters = nullptr;
  uint32_t* d_err = nullptr;
  uint32_t* h_err = nullptr;
  hipEvent_t err_copied = nullptr;
  bool err_pending = false;
  // After a device-side error has been reported the key is unusable: its
  // outputs since the failing launch are invalid and, for a 2DLASM sine that
  // could not be rounded, so is its generator state.
  bool dead = false;
  std::string dead_msg;
  uint32_t spin_limit = 1u << 21;  // group-barrier polls before giving up (about two seconds)
  cv::PlcmChain* d_chains = nullptr;
  std::vector<cv::PlcmChain> h_chains;  // host copy (tables of multi-stream batches)
  cv::LasmChain* d_lchains = nullptr;   // 2DLASM keys: generators of the bands
  std::vector<cv::LasmChain> h_lchains;
  // workspace, grown on demand
  uint32_t batch_frames = 0;
  uint8_t* d_ks = nullptr;
  uint8_t* d_scratch = nullptr;
  uint32_t* d_gm = nullptr;
  uint32_t* h_gm = nullptr;    // pinned staging of the shift tables
  size_t ws_frames = 0;
  hipEvent_t gm_done = nullptr;
  bool gm_pending = false;
  // launch shape
  uint32_t threads = 1024;
  uint32_t tile_enc = 0, tile_dec = 0;
  uint32_t max_band_rows = 0;
  size_t lds_max = 0;
  // graph replay of each batch's work (cv_launch.use_graph): one executable
  // graph per buffer set, least recently used dropped beyond kMaxGraphs
  bool use_graph = false;
  bool capturing = false;      // enqueueing into a capture: no events, no host state
  bool captured_err = false;   // the capture holds the error word's read-back
  hipStream_t cap = nullptr;   // private stream graphs are captured on
  struct GraphEntry {
    uint64_t sig[8];
    hipGraphExec_t exec;
    uint64_t last_use;
    bool reads_err;
  };
  static constexpr size_t kMaxGraphs = 16;
  std::vector<GraphEntry> graphs;
  uint64_t graph_clock = 0, graph_captures = 0, graph_replays = 0;
  // keystream lookahead (cv_launch.lookahead, PLCM keys): after each batch of
  // T frames, the next T frames' keystream is generated on a private stream
  // from a shadow copy of the generator states (two copies and two keystream
  // buffers, used in turn); the next batch takes it when it starts at the
  // predicted frame with the same T and the state was not set in between
  bool lookahead = false;
  struct Ahead {
    bool ready = false;                // events, shadow copies and chain tables set up
    SideStreams side;                  // private streams (default priority)
    hipEvent_t ks_ready = nullptr;     // call's stream: keystream ready, shadow states copied
    hipEvent_t done[2] = {};           // per shadow copy: the last lookahead using it is complete
    bool used[2] = {};
    double* d_shadow[2] = {};
    cv::PlcmChain* d_chains[2] = {};   // the key's chains with their states in shadow 0 / 1
    cv::LasmChain* d_lchains[2] = {};  // the same for a 2DLASM key
    uint8_t* d_ks[2] = {};
    size_t ks_cap[2] = {};
    bool valid = false;                // the fields below describe the last lookahead launched
    int target = -1, shadow = -1;      // its keystream buffer and shadow copy
    uint64_t frame_index = 0, epoch = 0;
    uint32_t T = 0;
  } ahead;
  uint64_t ahead_hits = 0, ahead_misses = 0;
  // Calls share the generator state and the workspace: the stream of the
  // key's last call that took a stream, and an event behind that call's work
  // (a call on another stream first waits for it).
  hipEvent_t order_ev = nullptr;
  hipStream_t order_stream = nullptr;
  bool order_has = false;
  // event profiling
  bool profiling = false;
  struct Span {
    hipEvent_t a, b;
    int kind;  // 0 = prbg, 1 = round
    uint64_t work;
  };
  std::vector<Span> spans;
  std::vector<hipEvent_t> event_pool;
  cv_profile prof{};
};

namespace cv {
namespace rt {

cv_status fail(cv_status s, const std::string& msg);
cv_status hip_fail(hipError_t e, const char* what);

#define CV_HIP(call)                                     \
  do {                                                   \
    hipError_t e_ = (call);                              \
    if (e_ != hipSuccess) return hip_fail(e_, #call);    \
  } while (0)

// Switch to the key's device for the lifetime of a call.
struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

// Row shifts of Eq. (1) for one frame, reduced mod W.
void shift_table(uint32_t H, uint32_t W, uint32_t s_c, uint32_t* gm);
bool aligned16(const void* p);
bool ranges_overlap(const void* a, size_t na, const void* b, size_t nb);
// Generator variant a launch of this key uses.
int prbg_variant(const cv_key* k);
// Largest pixel-word tile (rows) <= want accepted with `threads` threads.
uint32_t pw_tile_limit(const Geom& g, uint32_t threads, uint32_t want);
size_t lds_limit(int device);
cv_status check_async_errors(cv_key* k, bool wait);
// Chain steps of `frames` frames over all bands of the key.
uint64_t prbg_steps(const cv_key* k, uint64_t frames);
// Validates the buffers and seeds of an encrypt/decrypt call.
cv_status check_frames_args(const cv_key* k, const uint8_t* in, uint8_t* out, const uint32_t* s_c,
                            size_t n);
// Pixel-word LDS tile rows for geometry g with `threads` threads (0 = none).
uint32_t pw_tile_rows(const Geom& g, uint32_t threads, size_t lds_max);
// Encrypt or decrypt n frames of one key on its own path (plain or fused).
cv_status crypt_frames(cv_key* k, bool decrypt, const uint8_t* in, uint8_t* out,
                       const uint32_t* s_c, size_t n, void* stream);

// Keystream of T frames of one key into ks on st (either map), advancing it.
cv_status launch_keystream(cv_key* k, uint8_t* ks, uint32_t T, hipStream_t st);
cv_status queue_err_readback(cv_key* k, hipStream_t st);
// Sec. 3, Eq. (6): the admissible set of the 2DLASM control parameter.
bool lasm_mu_ok(double mu);
// Pixel-word kernels apply to this key and buffers with `threads` threads.
bool pw_eligible(const cv_key* k, const uint8_t* in, const uint8_t* out, uint32_t threads,
                 size_t lds_max);
// Key-path helpers (plain or fused rounds of one key, its workspace).
cv_status ensure_workspace(cv_key* k, size_t frames);
cv_status upload_shift_tables(cv_key* k, const uint32_t* s_c, size_t T, hipStream_t st);
// The private stream for work beside st (see SideStreams); release them.
cv_status side_stream(SideStreams& ss, int device, hipStream_t st, hipStream_t* out);
void side_streams_free(SideStreams& ss);
// Order a call of the key on st after its last call on another stream; after
// the call, note st and record the key's event there.
cv_status key_order_wait(const cv_key* k, hipStream_t st);
cv_status key_order_mark(cv_key* k, hipStream_t st);
cv_status run_rounds(cv_key* k, bool decrypt, const uint8_t* in, uint8_t* out, const uint8_t* ks,
                     uint32_t T, hipStream_t st);
// Pixel-word kernels apply to this key and these buffers.
bool use_pw(const cv_key* k, const uint8_t* in, const uint8_t* out, const uint8_t* ks);
// Groups a fused launch of this key and direction may use (resident capacity).
uint32_t fused_group_cap(const cv_key* k, bool decrypt);
// One fused launch over T frames on an explicit workspace (shift tables,
// exchange frames of `groups` groups, barrier counters, error word).
// `rows_tables` (T frames' tables of the row-run batch kernel, or null:
// then decryption with bands over one LDS tile takes the pixel-word kernel).
cv_status launch_fused_ws(const cv_key* k, bool decrypt, const uint8_t* in, uint8_t* out,
                          const uint8_t* ks, uint32_t T, const uint32_t* gm, uint8_t* fscratch,
                          uint32_t* counters, uint32_t* err, uint32_t groups, hipStream_t st,
                          uint8_t* rows_tables = nullptr);
// The byte round kernels over T frames on an explicit workspace (shift
// tables, one T-frame scratch buffer); `timed` records profiling events.
cv_status run_rounds_bytes_ws(cv_key* k, bool decrypt, const uint8_t* in, uint8_t* out,
                              const uint8_t* ks, uint32_t T, const uint32_t* gm, uint8_t* scratch,
                              hipStream_t st, bool timed);

// Work of one multi-stream tick.  Keystream locations are byte offsets from
// the tick's keystream base.
struct ChainJob {
  const cv_key* k;
  uint64_t ks_off;        // frame 0 of this key's keystream (canonical per-frame layout)
  uint64_t frame_stride;  // bytes from one frame's keystream to the next (0 = r*F)
  uint32_t frames;        // frames to generate (advances the key's generators)
};
struct FrameJob {
  const cv_key* k;
  const uint8_t* in;       // packed frame
  uint8_t* out;            // packed frame
  const uint8_t* in_last;  // last readable dword of the buffer `in` lies in
  uint64_t ks_off;         // this frame's keystream
  uint32_t s_c;            // confusion seed of this frame
  uint32_t decrypt;
};
// Enqueue keystream generation for `cj` and the rounds of `fj` (whose
// keystream is generated by this tick or was generated earlier) on st.
// Keystream offsets (ChainJob.ks_off, FrameJob.ks_off) count from ks_base;
// with a null ks_base they are device addresses.
// Every frame job must satisfy pw_eligible for the batch's shape.  With
// `hooks`, the work is launched kernel by kernel, and the hooks run on st
// between the keystream launches and the rounds launches, in this order:
// wait for each of `waits`, one launch of the state copies (sent with the
// tick's tables), record `ks_ready` (each if present).  The rounds launches
// then leave `reserve_cus` compute units of every XCD free (when at least a
// group's worth remain).
struct TickHooks {
  std::vector<hipEvent_t> waits;
  std::vector<cv::StateCopy> copies;
  hipEvent_t ks_ready = nullptr;
  uint32_t reserve_cus = 0;
};
cv_status batch_enqueue(cv_batch* b, const std::vector<ChainJob>& cj, const std::vector<FrameJob>& fj,
                        uint8_t* ks_base, hipStream_t st, const TickHooks* hooks = nullptr);
// Compute units of every XCD that the batch's rounds launches leave free
// (for work on other streams restricted to them).
void batch_set_reserve(cv_batch* b, uint32_t cus_per_xcd);
// Autotuner cache (tune_cache.cpp): the integer fields stored for a shape
// class in the file named by CV_TUNE_CACHE; false when absent (or no file).
bool tune_lookup(const std::string& key, std::map<std::string, int64_t>* fields);
bool tune_store(const std::string& key, const std::map<std::string, int64_t>& fields);
// Read-back of the batch's timeout flag as of its last completed tick.
bool batch_flag_set(const cv_batch* b);

}  // namespace rt
}  // namespace cv

namespace cv {
namespace crsin {
struct LdsTable;
}
namespace rt {
// The 2DLASM sine's tables for host evaluation (key schedule, cv_sin_stage1).
const crsin::LdsTable& crsin_host_table();
}  // namespace rt
}  // namespace cv
