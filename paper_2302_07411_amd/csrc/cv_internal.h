// Internal declarations of libchaosvid shared by the HIP kernels and the
// host runtime.  Not part of the public C ABI (that is include/chaosvid.h).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cv {

// Geometry of one video stream.  Band (subframe) i covers rows
// [floor(i*H/n), floor((i+1)*H/n)) -- Algorithm 2's band bounds,
// extended with floor so every row is covered when n does not divide H.
struct Geom {
  uint32_t H, W, C, n, r;
};

__host__ __device__ inline uint64_t band_lo(uint32_t H, uint32_t n, uint32_t i) {
  return ((uint64_t)i * H) / n;
}

// Band holding row `row`: the largest i with floor(i*H/n) <= row.
__host__ __device__ inline uint32_t band_of_row(uint32_t H, uint32_t n, uint32_t row) {
  return (uint32_t)((((uint64_t)row + 1) * n - 1) / H);
}

// ---------------------------------------------------------------- PRBG ----
// One chain = the two PLCMs of one band of one stream (Sec. 3).  Lane 2c of a
// wavefront iterates map 1 of chain c, lane 2c+1 map 2; 32 chains/wavefront.
struct PlcmChain {
  double* state;          // [2]: current x of map 1, map 2 (device, updated)
  double p[2];            // control parameters p of map 1, map 2
  double h[2];            // 1/2 - p, rounded once (bit-identical to forming it per step)
  double ip[2], ih[2];    // RN(1/p), RN(1/h) for the fast division path
  double lp[2], lh[2];    // RN(1/p - RN(1/p)), RN(1/h - RN(1/h)): low parts of the reciprocals
  uint64_t out_off;       // offset of this band's bytes in a frame's keystream
  uint64_t frame_stride;  // bytes from one frame's keystream to the next
  uint64_t nbytes;        // r * S_i bytes per frame
  uint32_t frames;        // frames of this chain when the launch passes n_frames = 0
  uint32_t pad;
};

// One band of a 2DLASM stream (Sec. 3, Eq. (6)): two maps, 12 bytes per step.
struct LasmChain {
  double* state;          // [4]: x, y of map 1, x, y of map 2 (device, updated)
  double mu[2];           // control parameters of map 1, map 2
  uint64_t out_off;       // offset of this band's bytes in a frame's keystream
  uint64_t frame_stride;  // bytes from one frame's keystream to the next
  uint64_t nbytes;        // r * S_i bytes per frame
  uint32_t frames;        // frames of this chain when the launch passes n_frames = 0
  uint32_t pad;
};

// 2DLASM keystream of n_frames frames (0: every chain its own `frames`); a
// sine whose rounding could not be decided stores 2 into *err.
// force_exact sends every sine to the exact path (for testing it).
hipError_t launch_prbg_lasm(const LasmChain* d_chains, uint32_t n_chains, uint8_t* ks_base,
                            uint32_t n_frames, uint32_t force_exact, uint32_t* err, hipStream_t s);
// The generator's correctly rounded sine on n device doubles in [0, RN(pi)].
hipError_t launch_cr_sin(const double* t, double* out, uint64_t n, uint32_t force_exact,
                         uint32_t* undecided, hipStream_t s);

// Generator variants (identical bytes): IEEE division; reciprocal division
// (valid only for chains that satisfy plcm_fast_ok); reciprocal division with
// one lane per piece of Eq. (5).
enum PrbgVariant : int {
  PRBG_EXACT = 0,
  PRBG_RECIP = 1,
  PRBG_RECIP_PAIR = 2,
  PRBG_SPEC = 3,        // two-operation quotient, verified and repaired by other wavefronts
  PRBG_SPEC_PLANT = 4,  // PRBG_SPEC with one-bit errors planted in the producer (testing)
};
constexpr int kPrbgVariants = 5;

// Generate n_frames frames of keystream for n_chains chains into ks_base
// (n_frames = 0: every chain generates its own `frames`).
hipError_t launch_prbg_plcm(const PlcmChain* d_chains, uint32_t n_chains, uint8_t* ks_base,
                            uint32_t n_frames, int variant, hipStream_t s);
// Workgroups of that launch.
uint32_t prbg_plcm_workgroups(uint32_t n_chains, int variant);

// Copy of `count` generator-state doubles from src to dst (device memory).
struct StateCopy {
  const double* src;
  double* dst;
  uint64_t count;
};
// One launch over n copies (a workgroup each).
hipError_t launch_copy_states(const StateCopy* d_copies, uint32_t n, hipStream_t s);

// Conditions under which the reciprocal division is exact for a whole orbit:
// p >= 2^-64 and the current state x is 0 or >= 2^-800.
inline bool plcm_fast_ok(double x, double p) {
  return p >= 0x1p-64 && (x == 0.0 || x >= 0x1p-800);
}

// --------------------------------------------------------------- rounds ---
// One confusion+diffusion round (or its inverse) over n_frames frames of one
// stream.  Frames, keystream and shift tables are laid out frame after frame.
struct RoundArgs {
  const uint8_t* src;     // round input, frame 0
  uint8_t* dst;           // round output, frame 0
  const uint8_t* ks;      // keystream of frame 0: band i's r*S_i bytes at r*lo_i*W*C
  const uint32_t* gm;     // per frame H entries: g(alpha) mod W
  uint64_t frame_bytes;   // F = H*W*C
  uint64_t ks_stride;     // keystream bytes per frame (r*F)
  Geom g;
  uint32_t j;             // round index 0..r-1
  uint32_t tile_rows;     // rows staged in LDS at a time
  uint32_t n_frames;
};

// Pixel-word rounds (C in {3,4}, W*C % 16 == 0, 16-byte aligned buffers):
// intermediate frames hold one 32-bit word per pixel.
struct RoundPwArgs {
  const uint8_t* src;     // round input, frame 0 (packed HWC or pixel words)
  uint8_t* dst;           // round output, frame 0 (packed HWC or pixel words)
  const uint8_t* ks;      // keystream of frame 0 (packed, canonical layout)
  const uint32_t* gm;     // per frame H entries: g(alpha) mod W
  Geom g;
  uint32_t j;
  uint32_t tile_rows;
  uint32_t n_frames;
  bool decrypt, src_packed, dst_packed;
};

size_t round_pw_lds_bytes(const Geom& g, uint32_t tile_rows);
hipError_t launch_round_pw(const RoundPwArgs& a, uint32_t threads, hipStream_t s);

// All r rounds of a batch of frames in one persistent launch (pixel-word
// layout conditions as above).  `scratch` holds two pixel-word frames per
// group, `counters` 128 bytes per group, `err` one word (left nonzero if a
// group barrier timed out or a group's workgroups ran on different XCDs).
struct RoundsFusedArgs {
  const uint8_t* in;
  uint8_t* out;
  const uint8_t* ks;
  const uint32_t* gm;
  uint8_t* scratch;
  uint32_t* counters;
  uint32_t* err;
  Geom g;
  uint32_t tile_rows, n_frames, groups, spin_limit;
  bool decrypt;
};

hipError_t launch_rounds_fused(const RoundsFusedArgs& a, uint32_t threads, hipStream_t s);
// Groups of n workgroups that can be resident at once (a multiple of 8; 0 if
// not even one group per XCD fits).
uint32_t rounds_fused_resident_groups(const Geom& g, uint32_t tile_rows, uint32_t threads,
                                      int device);

// All r encryption rounds of a batch of frames by whole source-row runs
// (rounds_skew.hip): the same arguments as launch_rounds_fused (decrypt must
// be false), tile rows from rounds_skew_tile_rows, 1024 threads per workgroup.
size_t rounds_skew_lds_bytes(const Geom& g, uint32_t tile_rows);
uint32_t rounds_skew_tile_rows(const Geom& g, size_t lds_max);  // 0: not applicable
uint32_t rounds_skew_resident_groups(const Geom& g, uint32_t tile_rows, int device);
hipError_t launch_rounds_skew(const RoundsFusedArgs& a, uint32_t tile_rows, hipStream_t s);

// All r decryption rounds of a batch of frames by whole source-row runs
// (rounds_unskew.hip): the same arguments as launch_rounds_fused (decrypt
// must be true), for geometries where every band fits the LDS as one tile.
bool rounds_unskew_applies(const Geom& g, size_t lds_max);
size_t rounds_unskew_lds_bytes(const Geom& g);
uint32_t rounds_unskew_resident_groups(const Geom& g, int device);
hipError_t launch_rounds_unskew(const RoundsFusedArgs& a, hipStream_t s);

// ------------------------------------------------------------- batch ----
// One (stream, frame) of a multi-stream tick.
struct BatchJob {
  const uint8_t* in;        // packed frame
  uint8_t* out;             // packed frame
  const uint8_t* in_last;   // last readable dword of the stream's input buffer
  const uint8_t* ks;        // this frame's keystream (canonical layout)
  const uint32_t* gm;       // this frame's g(alpha) mod W
  Geom g;
  uint32_t decrypt;
  uint32_t tile_rows;       // pixel-word tile rows for this geometry
  uint32_t tile_enc;        // row-run kernel: encryption tile rows (rounds_skew_tile_rows)
  uint32_t tile_dec;        // row-run kernel: decryption tile rows (batch_unskew_tile_rows)
};

// Workgroup slot of a batch launch: group | member << 12 | group size << 22
// (groups < 4096, sizes < 1024); kIdleSlot for a workgroup without a group.
// Workgroup i runs on XCD i % 8, so a group's slots all have one i % 8.
constexpr uint32_t kIdleSlot = 0xFFFFFFFFu;
__host__ __device__ inline uint32_t batch_slot(uint32_t group, uint32_t w, uint32_t G) {
  return group | (w << 12) | (G << 22);
}

struct BatchArgs {
  const BatchJob* jobs;
  const uint32_t* group_jobs;  // job indices, group after group
  const uint32_t* group_off;   // groups + 1 offsets into group_jobs
  const uint32_t* slots;       // n_slots entries, one per workgroup (batch_slot)
  uint8_t* scratch;            // per group two pixel-word frames of scratch_stride bytes
  uint64_t scratch_stride;
  uint32_t* counters;          // 128 bytes per group
  uint32_t* err;
  uint32_t n_slots, groups, spin_limit;
};

// rows = true: the row-run kernel (1024 threads; every job with tile_enc,
// tile_dec > 0); false: the pixel-word kernel.
// KQ: the row-run kernel's pixels per lane in the encryption diffusion (12
// for frame widths that are multiples of 12, else 4; 0: either, by each
// job's width, for a launch that holds both kinds).
hipError_t launch_batch_rounds(const BatchArgs& a, uint32_t C, uint32_t KQ, bool rows,
                               uint32_t threads, size_t lds, hipStream_t s);
// Workgroups per XCD that fit on the device at once; with `reserve_cus`, on
// all but that many compute units of every XCD, unless fewer than `min_wgs`
// would remain.
uint32_t batch_resident_slots(uint32_t C, uint32_t KQ, bool rows, uint32_t threads, size_t lds,
                              int device, uint32_t reserve_cus = 0, uint32_t min_wgs = 1);
// The row-run batch kernel over T frames of one stream (a single stream's
// decryption where a band exceeds one LDS tile).  Its tables -- T jobs, the
// group lists (group q takes frames q, q + groups, ...) and n_slots slots
// (groups of G workgroups, XCD-aware as above) -- are written into `tables`
// (stream_rows_table_bytes) by a kernel, so the launch reads no host memory.
struct StreamRows {
  BatchJob proto;          // frame 0's job; frame t's buffers are t frames further on
  uint64_t ks_stride;      // keystream bytes per frame
  uint32_t T, groups, G, KQ;
  size_t lds;              // batch_rows_lds_bytes of the job
  uint8_t* tables;
  uint8_t* scratch;        // two pixel-word frames per group
  uint32_t* counters;      // 128 bytes per group
  uint32_t* err;
  uint32_t spin_limit;
};
size_t stream_rows_table_bytes(uint32_t T, uint32_t n_slots);
uint32_t stream_rows_slots(uint32_t groups, uint32_t G);  // n_slots of a launch
hipError_t launch_stream_rows(const StreamRows& s, hipStream_t st);

// Row-run batch kernel: decryption tile rows for geometry g (0 = does not
// fit) and the LDS a job needs in either direction.
uint32_t batch_unskew_tile_rows(const Geom& g, size_t lds_max);
size_t batch_rows_lds_bytes(const Geom& g, bool decrypt, uint32_t tile_rows);

// LDS bytes a round kernel needs for a tile of `tile_rows` rows.
size_t round_lds_bytes(const Geom& g, uint32_t tile_rows);
hipError_t launch_round_enc(const RoundArgs& a, uint32_t threads, hipStream_t s);
hipError_t launch_round_dec(const RoundArgs& a, uint32_t threads, hipStream_t s);

}  // namespace cv
