// Confusion+diffusion rounds on pixel words, for 3- and 4-channel frames
// (Sec. 2, Eq. (1)-(4), Algorithm 2).
//
// Same computation as rounds.hip, laid out for gfx950's 32-bit datapath:
// between rounds a frame is kept as one 32-bit word per pixel (channel c in
// byte c, byte 3 zero for C = 3), so a confusion gather moves one aligned
// word per pixel, LDS tiles hold words, and diffusion runs on words.  Only
// the first round reads the caller's packed HWC bytes and only the last
// round writes packed bytes; the keystream stays packed (3 or 4 bytes per
// pixel) and is unpacked on load.
//
// Diffusion on a pixel word d (the pixel's D bytes, Eq. 3 unrolled):
// z = d ^ (d << 8); z ^= z << 16 gives byte c = d_0 ^ ... ^ d_c; XORing the
// running carry into all four bytes yields the cipher bytes, and byte 3
// (d_3 = 0 when C = 3) is exactly the carry into the next pixel.
//
// Requirements of this path (checked on the host): C in {3,4}, W a multiple
// of 16, all buffers 16-byte aligned, tiles of at most 16 pixels per thread.
#include "tile_ops.h"

namespace cv {
namespace {

using namespace tile;

struct PwArgs {
  const uint8_t* src;
  uint8_t* dst;
  const uint8_t* src_last;  // last readable dword of the whole source buffer
  const uint8_t* ks;
  const uint32_t* gm;
  uint64_t src_stride, dst_stride, ks_stride;  // bytes per frame
  Geom g;
  uint32_t j, tile_rows, n_frames;
};

__device__ __forceinline__ View frame_view(const PwArgs& A, uint32_t f) {
  View v;
  v.src = A.src + (uint64_t)f * A.src_stride;
  v.dst = A.dst + (uint64_t)f * A.dst_stride;
  v.src_last = A.src_last;
  v.ks = A.ks + (uint64_t)f * A.ks_stride;
  v.gm = A.gm + (uint64_t)f * A.g.H;
  return v;
}

template <uint32_t C, bool kSrcPacked, bool kDstPacked>
__global__ __launch_bounds__(kMaxThreads) void round_enc_pw_kernel(PwArgs A) {
  extern __shared__ __align__(16) uint32_t tile[];
  __shared__ uint32_t scan_sh[kMaxThreads / 64];
  const uint32_t band = blockIdx.x, f = blockIdx.y;
  const View v = frame_view(A, f);
  const uint32_t lo = (uint32_t)band_lo(A.g.H, A.g.n, band), hi = (uint32_t)band_lo(A.g.H, A.g.n, band + 1);
  uint32_t carry = enc_seed<C, kSrcPacked>(v, A.g, band);
  for (uint32_t t0 = lo; t0 < hi; t0 += A.tile_rows)
    carry = enc_tile<C, kSrcPacked, kDstPacked>(v, A.g, A.j, lo, hi, t0, min(A.tile_rows, hi - t0),
                                                 carry, tile, scan_sh);
}

template <uint32_t C, bool kSrcPacked, bool kDstPacked>
__global__ __launch_bounds__(kMaxThreads) void round_dec_pw_kernel(PwArgs A) {
  extern __shared__ __align__(16) uint32_t tile[];
  const uint32_t f = blockIdx.y;
  const View v = frame_view(A, f);
  uint32_t* blo = tile + (size_t)A.tile_rows * A.g.W;
  uint32_t* seed = blo + A.g.n + 1;
  dec_seeds<C, kSrcPacked>(v, A.g, A.j, blo, seed);
  const uint32_t t0 = blockIdx.x * A.tile_rows;
  dec_tile<C, kSrcPacked, kDstPacked>(v, A.g, A.j, t0, min(A.tile_rows, A.g.H - t0), tile, blo, seed);
}

template <uint32_t C>
hipError_t launch_pw(bool decrypt, bool src_packed, bool dst_packed, const PwArgs& a,
                     uint32_t threads, size_t lds, dim3 grid, hipStream_t s) {
#define CV_PW_LAUNCH(K, SP, DP) \
  hipLaunchKernelGGL((K<C, SP, DP>), grid, dim3(threads), lds, s, a)
  if (!decrypt) {
    if (src_packed && dst_packed) CV_PW_LAUNCH(round_enc_pw_kernel, true, true);
    else if (src_packed) CV_PW_LAUNCH(round_enc_pw_kernel, true, false);
    else if (dst_packed) CV_PW_LAUNCH(round_enc_pw_kernel, false, true);
    else CV_PW_LAUNCH(round_enc_pw_kernel, false, false);
  } else {
    if (src_packed && dst_packed) CV_PW_LAUNCH(round_dec_pw_kernel, true, true);
    else if (src_packed) CV_PW_LAUNCH(round_dec_pw_kernel, true, false);
    else if (dst_packed) CV_PW_LAUNCH(round_dec_pw_kernel, false, true);
    else CV_PW_LAUNCH(round_dec_pw_kernel, false, false);
  }
#undef CV_PW_LAUNCH
  return hipGetLastError();
}

// ------------------------------------------------------ fused r rounds ---
// One launch runs all r rounds of a batch of frames (Algorithm 1's round
// loop without returning to the host).  Workgroups form groups of n, one per
// band; a group walks frames f = group, group + G, ...  Each round a
// workgroup writes its band to the group's pixel-word scratch, then the
// group meets at a barrier (device-scope release/acquire on a counter that
// only the group's n workgroups touch) before the next round reads the whole
// frame.  The group's workgroups are placed on one XCD (workgroup i is
// dispatched to XCD i mod 8), so the exchange goes through that XCD's L2:
// releasing needs only each wavefront's stores to have reached L2 (no
// device-wide L2 write-back), and acquiring is one device-scope cache
// invalidate per workgroup after the wait (a workgroup-scope invalidate is
// not enough: it leaves the CU's L1 lines, rewritten by other CUs, valid).
// That holds only if every member really runs on the same XCD, so each
// workgroup reads its XCC id at start and records it for its group; a
// member on another XCD raises `err` before any exchange happens.
// A barrier wait is bounded too: after `spin_limit` polls the workgroup
// raises `err` and leaves, so a launch that cannot keep a group resident
// ends instead of hanging.  The host reports `err` as an error.
struct FusedArgs {
  const uint8_t* in;        // packed input frames
  uint8_t* out;             // packed output frames
  const uint8_t* in_last;   // last readable dword of `in`
  const uint8_t* ks;        // keystream (packed, canonical), frame after frame
  const uint32_t* gm;       // shift tables, H per frame
  uint8_t* scratch;         // per group: two pixel-word frames
  uint32_t* counters;       // per group one 128-byte line: [0] barrier counter (zero at
                            // launch), [1] XCC id of the group (all ones at launch)
  uint32_t* err;            // set to 1 when a barrier wait times out
  Geom g;
  uint32_t tile_rows, n_frames, groups, spin_limit;
  bool decrypt;
};

template <uint32_t C>
__global__ __launch_bounds__(kMaxThreads) void rounds_fused_kernel(FusedArgs A) {
  extern __shared__ __align__(16) uint32_t tile[];
  __shared__ uint32_t scan_sh[kMaxThreads / 64];
  const Geom g = A.g;
  // XCD-aware placement: workgroup i runs on XCD i % 8; group members share it
  const uint32_t i = blockIdx.x, xcd = i % 8, idx = i / 8;
  const uint32_t group = xcd + 8 * (idx / g.n), band = idx % g.n;
  if (group >= A.groups) return;
  const uint64_t pwf = (uint64_t)g.H * g.W * 4, F = (uint64_t)g.H * g.W * C;
  uint8_t* buf[2] = {A.scratch + (uint64_t)group * 2 * pwf, A.scratch + (uint64_t)group * 2 * pwf + pwf};
  uint32_t* ctr = A.counters + 32 * group;
  check_group_xcc(ctr + 1, A.err);
  uint32_t* blo = tile + (size_t)A.tile_rows * g.W;
  uint32_t* seed = blo + g.n + 1;
  const uint32_t lo = (uint32_t)band_lo(g.H, g.n, band), hi = (uint32_t)band_lo(g.H, g.n, band + 1);
  uint32_t nbar = 0;
  for (uint32_t f = group; f < A.n_frames; f += A.groups) {
    View v;
    v.ks = A.ks + (uint64_t)f * g.r * F;
    v.gm = A.gm + (uint64_t)f * g.H;
    for (uint32_t s = 0; s < g.r; s++) {
      const bool first = s == 0, last = s + 1 == g.r;
      v.src = first ? A.in + (uint64_t)f * F : buf[(s + 1) & 1];
      v.src_last = first ? A.in_last : buf[(s + 1) & 1] + pwf - 4;
      v.dst = last ? A.out + (uint64_t)f * F : buf[s & 1];
      if (!A.decrypt) {
        const uint32_t j = s;
        uint32_t carry = first ? enc_seed<C, true>(v, g, band) : enc_seed<C, false>(v, g, band);
        for (uint32_t t0 = lo; t0 < hi; t0 += A.tile_rows) {
          const uint32_t R = min(A.tile_rows, hi - t0);
          if (first && last) carry = enc_tile<C, true, true>(v, g, j, lo, hi, t0, R, carry, tile, scan_sh);
          else if (first) carry = enc_tile<C, true, false>(v, g, j, lo, hi, t0, R, carry, tile, scan_sh);
          else if (last) carry = enc_tile<C, false, true>(v, g, j, lo, hi, t0, R, carry, tile, scan_sh);
          else carry = enc_tile<C, false, false>(v, g, j, lo, hi, t0, R, carry, tile, scan_sh);
          __syncthreads();  // the next tile's gather overwrites LDS
        }
      } else {
        const uint32_t j = g.r - 1 - s;
        if (first) dec_seeds<C, true>(v, g, j, blo, seed);
        else dec_seeds<C, false>(v, g, j, blo, seed);
        for (uint32_t t0 = lo; t0 < hi; t0 += A.tile_rows) {
          const uint32_t R = min(A.tile_rows, hi - t0);
          if (first && last) dec_tile<C, true, true>(v, g, j, t0, R, tile, blo, seed);
          else if (first) dec_tile<C, true, false>(v, g, j, t0, R, tile, blo, seed);
          else if (last) dec_tile<C, false, true>(v, g, j, t0, R, tile, blo, seed);
          else dec_tile<C, false, false>(v, g, j, t0, R, tile, blo, seed);
        }
      }
      // every band of this round is written before any band of the next
      // round (or the next frame's first round, which reuses the scratch)
      nbar++;
      if (!group_barrier(ctr, nbar * g.n, A.spin_limit, A.err)) return;
    }
  }
}

// Per-launch reset of the group lines: counter 0, XCC slot all ones.
__global__ void reset_groups(uint32_t* p, uint32_t groups) {
  for (uint32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < groups; k += gridDim.x * blockDim.x) {
    p[32 * k] = 0;
    p[32 * k + 1] = 0xFFFFFFFFu;
  }
}

}  // namespace

size_t round_pw_lds_bytes(const Geom& g, uint32_t tile_rows) {
  return (size_t)tile_rows * g.W * 4 + 8 * ((size_t)g.n + 1) + 16;
}

hipError_t launch_round_pw(const RoundPwArgs& r, uint32_t threads, hipStream_t s) {
  PwArgs a;
  a.src = r.src;
  a.dst = r.dst;
  a.ks = r.ks;
  a.gm = r.gm;
  a.g = r.g;
  a.j = r.j;
  a.tile_rows = r.tile_rows;
  a.n_frames = r.n_frames;
  const uint64_t pw = (uint64_t)r.g.H * r.g.W * 4, packed = (uint64_t)r.g.H * r.g.W * r.g.C;
  a.src_stride = r.src_packed ? packed : pw;
  a.dst_stride = r.dst_packed ? packed : pw;
  a.ks_stride = (uint64_t)r.g.r * packed;
  a.src_last = r.src + (uint64_t)r.n_frames * a.src_stride - 4;
  const size_t lds = round_pw_lds_bytes(r.g, r.tile_rows);
  dim3 grid = r.decrypt ? dim3((r.g.H + r.tile_rows - 1) / r.tile_rows, r.n_frames)
                        : dim3(r.g.n, r.n_frames);
  if (r.g.C == 3) return launch_pw<3>(r.decrypt, r.src_packed, r.dst_packed, a, threads, lds, grid, s);
  return launch_pw<4>(r.decrypt, r.src_packed, r.dst_packed, a, threads, lds, grid, s);
}

}  // namespace cv

namespace cv {

hipError_t launch_rounds_fused(const RoundsFusedArgs& r, uint32_t threads, hipStream_t s) {
  FusedArgs a;
  a.in = r.in;
  a.out = r.out;
  const uint64_t F = (uint64_t)r.g.H * r.g.W * r.g.C;
  a.in_last = r.in + (uint64_t)r.n_frames * F - 4;
  a.ks = r.ks;
  a.gm = r.gm;
  a.scratch = r.scratch;
  a.counters = r.counters;
  a.err = r.err;
  a.g = r.g;
  a.tile_rows = r.tile_rows;
  a.n_frames = r.n_frames;
  a.groups = r.groups;
  a.spin_limit = r.spin_limit;
  a.decrypt = r.decrypt;
  // per launch: counters zero, XCC slots all ones (a kernel, not a memset)
  hipLaunchKernelGGL(reset_groups, dim3(1), dim3(256), 0, s, r.counters, r.groups);
  const size_t lds = round_pw_lds_bytes(r.g, r.tile_rows);
  // groups rounded up to a multiple of 8 so that group members share an XCD
  const uint32_t slots = ((r.groups + 7) / 8) * 8 * r.g.n;
  if (r.g.C == 3)
    hipLaunchKernelGGL(rounds_fused_kernel<3>, dim3(slots), dim3(threads), lds, s, a);
  else
    hipLaunchKernelGGL(rounds_fused_kernel<4>, dim3(slots), dim3(threads), lds, s, a);
  return hipGetLastError();
}

uint32_t rounds_fused_resident_groups(const Geom& g, uint32_t tile_rows, uint32_t threads,
                                      int device) {
  int per_cu = 0, cus = 0;
  const size_t lds = round_pw_lds_bytes(g, tile_rows);
  hipError_t e = g.C == 3 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(
                                &per_cu, rounds_fused_kernel<3>, threads, lds)
                          : hipOccupancyMaxActiveBlocksPerMultiprocessor(
                                &per_cu, rounds_fused_kernel<4>, threads, lds);
  if (e != hipSuccess || per_cu <= 0) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess) return 0;
  const uint32_t per_xcd = (uint32_t)per_cu * (uint32_t)cus / 8;  // workgroup slots per XCD
  return (per_xcd / g.n) * 8;                                     // groups that fit, 8 XCDs
}

}  // namespace cv
