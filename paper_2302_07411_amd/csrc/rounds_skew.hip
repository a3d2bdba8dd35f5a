// All r encryption rounds of a batch of frames (Sec. 2, Eq. (1) and (3),
// Algorithm 1's round loop), with the confusion gather done as whole source
// row runs and the diffusion done on packed bytes (the per-tile steps are in
// skew_ops.h).  Between rounds a frame is kept as pixel words in the group's
// scratch; the last round writes packed bytes.
//
// Workgroups form groups of n (one per band) that walk frames and meet at a
// barrier after every round, as in the pixel-word fused kernel; the whole
// band (or the largest tile of rows that fits the LDS) is processed at once.
#include "skew_ops.h"

namespace cv {
namespace {

using namespace skew;

struct SkewArgs {
  const uint8_t* in;       // packed input frames
  uint8_t* out;            // packed output frames
  const uint8_t* in_last;  // last readable dword of `in`
  const uint8_t* ks;       // keystream (packed, canonical), frame after frame
  const uint32_t* gm;      // shift tables g(alpha) mod W, H per frame
  uint8_t* scratch;        // per group: two pixel-word frames
  uint32_t* counters;      // per group one 128-byte line: barrier counter, XCC id
  uint32_t* err;
  Geom g;
  uint32_t tile_rows, n_frames, groups, spin_limit;
};

template <uint32_t C, uint32_t KQ, bool kFull>
__global__ __launch_bounds__(kThreads) void rounds_skew_kernel(SkewArgs A) {
  extern __shared__ __align__(16) uint32_t lds[];
  __shared__ uint32_t wsum[kWaves];
  const Geom g = A.g;
  // XCD-aware placement: workgroup i runs on XCD i % 8; group members share it
  const uint32_t i = blockIdx.x, xcd = i % 8, idx = i / 8;
  const uint32_t group = xcd + 8 * (idx / g.n), band = idx % g.n;
  if (group >= A.groups) return;
  const uint64_t pwf = (uint64_t)g.H * g.W * 4, F = (uint64_t)g.H * g.W * C;
  uint8_t* buf[2] = {A.scratch + (uint64_t)group * 2 * pwf, A.scratch + (uint64_t)group * 2 * pwf + pwf};
  uint32_t* ctr = A.counters + 32 * group;
  check_group_xcc(ctr + 1, A.err);
  const uint32_t lo = (uint32_t)band_lo(g.H, g.n, band), hi = (uint32_t)band_lo(g.H, g.n, band + 1);
  uint32_t nbar = 0;
  for (uint32_t f = group; f < A.n_frames; f += A.groups) {
    View v;
    v.ks = A.ks + (uint64_t)f * g.r * F;
    v.gm = A.gm + (uint64_t)f * g.H;
    // the seed of this band (Eq. 3): the last byte of band (band+1) mod n
    // after confusion, i.e. source pixel (a, o) of Eq. (1) for the last
    // position of that band; the same position in every round of the frame
    const int64_t seed_at = (int64_t)enc_seed_index(v, g, band);
    for (uint32_t s = 0; s < g.r; s++) {
      const bool first = s == 0, last = s + 1 == g.r;
      v.src = first ? A.in + (uint64_t)f * F : buf[(s + 1) & 1];
      v.src_last = first ? A.in_last : buf[(s + 1) & 1] + pwf - 4;
      v.dst = last ? A.out + (uint64_t)f * F : buf[s & 1];
      uint32_t carry = 0;
      for (uint32_t t0 = lo; t0 < hi; t0 += A.tile_rows) {
        const uint32_t R = min(A.tile_rows, hi - t0);
        const int64_t sa = t0 == lo ? seed_at : -1;
        if (first && last)
          carry = skew_tile<C, KQ, true, true, kFull>(v, g, s, lo, hi, t0, R, carry, sa, lds, wsum);
        else if (first)
          carry = skew_tile<C, KQ, true, false, kFull>(v, g, s, lo, hi, t0, R, carry, sa, lds, wsum);
        else if (last)
          carry = skew_tile<C, KQ, false, true, kFull>(v, g, s, lo, hi, t0, R, carry, sa, lds, wsum);
        else
          carry = skew_tile<C, KQ, false, false, kFull>(v, g, s, lo, hi, t0, R, carry, sa, lds, wsum);
        __syncthreads();  // the next tile's gather overwrites the LDS tile and wsum
      }
      nbar++;
      if (!group_barrier(ctr, nbar * g.n, A.spin_limit, A.err)) return;
    }
  }
}

__global__ void reset_skew_groups(uint32_t* p, uint32_t groups) {
  for (uint32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < groups; k += gridDim.x * blockDim.x) {
    p[32 * k] = 0;
    p[32 * k + 1] = 0xFFFFFFFFu;
  }
}

template <uint32_t C, uint32_t KQ, bool kFull>
const void* skew_fn() {
  return reinterpret_cast<const void*>(&rounds_skew_kernel<C, KQ, kFull>);
}

const void* pick(const Geom& g) {
  const bool full = g.W % g.H == 0;
  const bool q12 = g.W % 12 == 0;
  if (g.C == 3) {
    if (q12) return full ? skew_fn<3, 12, true>() : skew_fn<3, 12, false>();
    return full ? skew_fn<3, 4, true>() : skew_fn<3, 4, false>();
  }
  if (q12) return full ? skew_fn<4, 12, true>() : skew_fn<4, 12, false>();
  return full ? skew_fn<4, 4, true>() : skew_fn<4, 4, false>();
}

}  // namespace

size_t rounds_skew_lds_bytes(const Geom& g, uint32_t tile_rows) {
  return (size_t)tile_rows * (g.W + kRowPad) * 4;
}

uint32_t rounds_skew_tile_rows(const Geom& g, size_t lds_max) {
  if (!((g.C == 3 || g.C == 4) && g.W % 16 == 0)) return 0;
  const size_t reserve = 1024;  // static LDS of the kernel and group-barrier words
  if (lds_max <= reserve) return 0;
  uint32_t rows = (uint32_t)((lds_max - reserve) / ((size_t)(g.W + kRowPad) * 4));
  rows = std::min<uint32_t>(rows, kMaxTilePix / g.W);
  uint32_t band_max = 0;
  for (uint32_t i = 0; i < g.n; i++)
    band_max = std::max<uint32_t>(band_max, (uint32_t)(band_lo(g.H, g.n, i + 1) - band_lo(g.H, g.n, i)));
  rows = std::min(rows, band_max);
  const uint32_t M = (g.W + g.H - 1) / g.H;
  if (rows * M > kThreads) rows = kThreads / M;
  return rows;
}

uint32_t rounds_skew_resident_groups(const Geom& g, uint32_t tile_rows, int device) {
  if (tile_rows == 0) return 0;
  int per_cu = 0, cus = 0;
  const size_t lds = rounds_skew_lds_bytes(g, tile_rows);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, pick(g), kThreads, lds) != hipSuccess ||
      per_cu <= 0)
    return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess) return 0;
  const uint32_t per_xcd = (uint32_t)per_cu * (uint32_t)cus / 8;
  return (per_xcd / g.n) * 8;
}

hipError_t launch_rounds_skew(const RoundsFusedArgs& r, uint32_t tile_rows, hipStream_t s) {
  SkewArgs a;
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
  a.tile_rows = tile_rows;
  a.n_frames = r.n_frames;
  a.groups = r.groups;
  a.spin_limit = r.spin_limit;
  hipLaunchKernelGGL(reset_skew_groups, dim3(1), dim3(256), 0, s, r.counters, r.groups);
  const size_t lds = rounds_skew_lds_bytes(r.g, tile_rows);
  const uint32_t slots = ((r.groups + 7) / 8) * 8 * r.g.n;
  const void* fn = pick(r.g);
  if (lds > 64 * 1024) {
    const hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  void* args[] = {&a};
  return hipLaunchKernel(fn, dim3(slots), dim3(kThreads), args, lds, s);
}

}  // namespace cv
