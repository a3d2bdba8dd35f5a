// All r encryption rounds of a batch of frames (Sec. 2, Eq. (1) and (3),
// Algorithm 1's round loop), with the confusion gather done as whole source
// row runs and the diffusion done on packed bytes.
//
// Eq. (1) sends source pixel (a, o) to row alpha = (a+o) mod H, column
// beta = (o + g(alpha)) mod W.  Seen from a block of destination rows
// [t0, t0+R), it is a column skew followed by one rotation per row: the tile
// T[k][o] (k = alpha - t0) holds source pixel ((t0+k-o) mod H, o), and row k
// of the result is row k of T rotated right by g(t0+k).  For a fixed source
// row a, the pixels that land in the tile are the R consecutive columns
// o = (t0+k-a) mod H (plus multiples of H when W > H), so the gather reads
// each source row as a contiguous run: one coalesced load instruction covers
// most of a run, and consecutive lanes write T[k][o] at LDS words that step
// by W+kRowPad+1, i.e. across banks.  The rotation is applied when the tile is
// read: row k starts at LDS word rowbase(k) = k*(W+kRowPad) + (g mod 4), so
// the four pixels at beta, beta+1, ... (beta a multiple of 4) sit at one
// 16-byte aligned address, and three copied words after each row cover reads
// that wrap past column W-1.
//
// Diffusion (Eq. 3) runs in chain order over bytes: each lane takes KQ
// consecutive pixels of a row (KQ*C bytes, KQ*C/4 words), packs the tile's
// pixel words into byte order with byte permutes, forms D = b ^ (Y + b) per
// byte, and XOR-prefixes the words (shift-XOR within a word, the previous
// word's last byte broadcast into the next).  Lane carries come from a DPP
// scan of lane totals inside the wavefront; wavefronts own consecutive
// stretches of runs, so one block scan of 16 wavefront totals per tile
// completes the chain.  Between rounds a frame is kept as pixel words in the
// group's scratch; the last round writes packed bytes.
//
// Workgroups form groups of n (one per band) that walk frames and meet at a
// barrier after every round, as in the pixel-word fused kernel; the whole
// band (or the largest tile of rows that fits the LDS) is processed at once.
#include "tile_ops.h"

namespace cv {
namespace {

using namespace tile;

constexpr uint32_t kThreads = 1024;
constexpr uint32_t kWaves = kThreads / 64;
constexpr uint32_t kRowPad = 8;      // per LDS row: 3 wrap words + up to 3 alignment words
constexpr uint32_t kMaxTilePix = 36 * kThreads;  // pixels of a tile: at most 36 per thread
// source rows in flight per thread in the gather (measured at 768x768x3: 8
// is fastest; 16 gains nothing, 24 spills registers)
constexpr uint32_t kGatherBatch = 8;

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

__device__ __forceinline__ uint32_t rowbase(uint32_t k, uint32_t W, uint32_t gk) {
  return k * (W + kRowPad) + (gk & 3u);
}

// Inclusive XOR scan across the 64 lanes of a wavefront (DPP row shifts, then
// row broadcasts).
__device__ __forceinline__ uint32_t wave_xor_incl(uint32_t x) {
  x ^= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xF, 0xF, false);  // row_shr:1
  x ^= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xF, 0xF, false);  // row_shr:2
  x ^= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xF, 0xF, false);  // row_shr:4
  x ^= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xF, 0xF, false);  // row_shr:8
  x ^= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xA, 0xF, false);  // row_bcast:15
  x ^= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x143, 0xC, 0xF, false);  // row_bcast:31
  return x;
}

__device__ __forceinline__ uint32_t bcast_top(uint32_t z) {  // byte 3 into all four bytes
  return __builtin_amdgcn_perm(z, z, 0x07070707u);
}

// Confusion gather of tile rows [t0, t0+R) into T (see the file comment).
template <uint32_t C, bool kSrcPacked, bool kFull, uint32_t kU>
__device__ __forceinline__ void skew_gather(const View& v, const Geom& g, uint32_t t0, uint32_t R,
                                            uint32_t* lds) {
  const uint32_t W = g.W, H = g.H;
  const uint32_t M = (W + H - 1) / H;  // runs per source row
  const uint32_t per = R * M;
  const uint32_t A = kThreads / per;   // source rows walked side by side
  const uint32_t t = threadIdx.x;
  if (t >= per * A) return;
  const uint32_t k = t % R, rest = t / R, m = rest % M, s = rest / M;
  const uint32_t rb = rowbase(k, W, v.gm[t0 + k]) + m * H;
  const uint32_t mH = m * H;
  // every load of a batch is issued before the first LDS write, so the
  // gather costs about one memory round trip per batch of kU source rows
  for (uint32_t a0 = s; a0 < H; a0 += kU * A) {
    uint32_t val[kU];
#pragma unroll
    for (uint32_t u = 0; u < kU; u++) {
      const uint32_t a = a0 + u * A;
      const int32_t d = (int32_t)(t0 + k) - (int32_t)a;  // alpha - a
      const uint32_t orel = d < 0 ? (uint32_t)(d + (int32_t)H) : (uint32_t)d;
      const bool ok = a < H && (kFull || orel + mH < W);
      val[u] = src_pixel<C, kSrcPacked>(v, ok ? a * W + orel + mH : 0u);
    }
#pragma unroll
    for (uint32_t u = 0; u < kU; u++) {
      const uint32_t a = a0 + u * A;
      const int32_t d = (int32_t)(t0 + k) - (int32_t)a;
      const uint32_t orel = d < 0 ? (uint32_t)(d + (int32_t)H) : (uint32_t)d;
      if (a < H && (kFull || orel + mH < W)) lds[rb + orel] = val[u] & pixel_mask<C>();
    }
  }
}

// One tile of one round: gather, diffusion seeded with `carry`, store.
// Returns the carry into the next tile of the band.
// `seed_at` >= 0: the tile starts the band, and its carry is the diffusion
// seed, byte C-1 of source pixel seed_at (loaded here, before the gather);
// otherwise `carry` comes from the previous tile.
template <uint32_t C, uint32_t KQ, bool kSrcPacked, bool kDstPacked, bool kFull>
__device__ uint32_t skew_tile(const View& v, const Geom& g, uint32_t j, uint32_t lo, uint32_t hi,
                              uint32_t t0, uint32_t R, uint32_t carry, int64_t seed_at,
                              uint32_t* lds, uint32_t* wsum) {
  constexpr uint32_t DW = KQ * C / 4;           // words per run in byte order
  constexpr uint32_t NP = kMaxTilePix / (KQ * kThreads);  // passes per wavefront, at most
  const uint32_t W = g.W;
  const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
  const uint32_t rpr = W / KQ;                  // runs per row
  const uint32_t nruns = R * rpr;
  const uint32_t np = (nruns + kThreads - 1) / kThreads;  // passes (<= NP)
  const uint64_t S = (uint64_t)(hi - lo) * W * C;
  const uint8_t* kt = v.ks + (uint64_t)g.r * lo * W * C + (uint64_t)j * S + (uint64_t)(t0 - lo) * W * C;
  // the band's seed pixel: its latency hides behind the gather
  if (seed_at >= 0) carry = (src_pixel<C, kSrcPacked>(v, (uint64_t)seed_at) >> (8 * (C - 1))) & 0xFFu;
  skew_gather<C, kSrcPacked, kFull, kGatherBatch>(v, g, t0, R, lds);
  __syncthreads();
  // wrap words: columns 0..2 of every row again after column W-1 (a tile
  // of narrow rows can have more than kThreads/3 rows)
  for (uint32_t x = threadIdx.x; x < 3 * R; x += kThreads) {
    const uint32_t k = x / 3, o = x % 3;
    const uint32_t rb = rowbase(k, W, v.gm[t0 + k]);
    lds[rb + W + o] = lds[rb + o];
  }
  __syncthreads();

  uint32_t Z[NP][DW];
  uint32_t pass_excl[NP];  // this lane's carry within its wavefront's stretch, per pass
  uint32_t wave_total = 0;
#pragma unroll
  for (uint32_t p = 0; p < NP; p++) {
    const uint32_t q = (wave * np + p) * 64 + lane;  // run index: wavefronts own stretches
    const bool ok = p < np && q < nruns;
    uint32_t P[DW], K[DW];
    {
      // the run's keystream words by 16-byte loads (a lane's KQ*C bytes are
      // only 4-byte aligned); lanes without a run read run 0 and drop it
      const uint8_t* kp = kt + (uint64_t)(ok ? q : 0u) * KQ * C;
#pragma unroll
      for (uint32_t i = 0; i + 4 <= DW; i += 4) {
        const v4u32a4 w = gload4u(kp + 4 * i);
        K[i] = w.x;
        K[i + 1] = w.y;
        K[i + 2] = w.z;
        K[i + 3] = w.w;
      }
#pragma unroll
      for (uint32_t i = DW / 4 * 4; i < DW; i++) K[i] = g32(kp)[i];
#pragma unroll
      for (uint32_t i = 0; i < DW; i++) K[i] = ok ? K[i] : 0u;
    }
    if (ok) {
      const uint32_t k = q / rpr, b0 = (q - k * rpr) * KQ;
      const uint32_t gk = v.gm[t0 + k];
      const uint32_t rb = rowbase(k, W, gk);
#pragma unroll
      for (uint32_t i = 0; i < KQ / 4; i++) {
        int32_t x = (int32_t)(b0 + 4 * i) - (int32_t)gk;
        if (x < 0) x += (int32_t)W;
        const uint4 y = *reinterpret_cast<const uint4*>(lds + rb + (uint32_t)x);
        const uint32_t w4[4] = {y.x, y.y, y.z, y.w};
        if constexpr (C == 3) {
          pack4(w4, P + 3 * i);
        } else {
#pragma unroll
          for (uint32_t e = 0; e < 4; e++) P[4 * i + e] = w4[e];
        }
      }
    } else {
#pragma unroll
      for (uint32_t i = 0; i < DW; i++) P[i] = 0;
    }
    // D = b ^ (Y + b) per byte, then the XOR prefix over the run's bytes
    uint32_t run = 0;  // broadcast of the last byte so far
#pragma unroll
    for (uint32_t i = 0; i < DW; i++) {
      uint32_t z = K[i] ^ add_bytes(P[i], K[i]);
      z ^= z << 8;
      z ^= z << 16;
      z ^= run;
      run = bcast_top(z);
      Z[p][i] = z;
    }
    const uint32_t tot = Z[p][DW - 1] >> 24;     // XOR of all bytes of the run
    const uint32_t incl = wave_xor_incl(tot);
    pass_excl[p] = (incl ^ tot ^ wave_total) & 0xFFu;
    wave_total ^= (uint32_t)__builtin_amdgcn_readlane((int)incl, 63);
  }
  if (lane == 0) wsum[wave] = wave_total & 0xFFu;
  __syncthreads();
  const uint32_t wl = lane < kWaves ? wsum[lane] : 0u;
  const uint32_t wincl = wave_xor_incl(wl);
  const uint32_t before = wave == 0 ? 0u : (uint32_t)__builtin_amdgcn_readlane((int)wincl, (int)wave - 1);
  const uint32_t all = (uint32_t)__builtin_amdgcn_readlane((int)wincl, kWaves - 1);
  // Stores staged through the tile (free: every wavefront has read it before
  // the block scan's barrier; run q's output words go to words [q*OW, (q+1)*OW),
  // within the tile since q*KQ is a pixel of it), so that each store
  // instruction writes 1 KB of consecutive bytes.
  constexpr uint32_t OW = kDstPacked ? DW : KQ;   // output words per run
#pragma unroll
  for (uint32_t p = 0; p < NP; p++) {
    const uint32_t q = (wave * np + p) * 64 + lane;
    if (!(p < np && q < nruns)) continue;
    const uint32_t c = ((carry ^ before ^ pass_excl[p]) & 0xFFu) * 0x01010101u;
    uint32_t out[DW];
#pragma unroll
    for (uint32_t i = 0; i < DW; i++) out[i] = Z[p][i] ^ c;
    uint32_t* st = lds + q * OW;
    if constexpr (kDstPacked) {
#pragma unroll
      for (uint32_t i = 0; i < DW; i++) st[i] = out[i];
    } else {
#pragma unroll
      for (uint32_t i = 0; i < KQ / 4; i++) {
        uint32_t w4[4];
        if constexpr (C == 3) {
          unpack4(out + 3 * i, w4);
        } else {
#pragma unroll
          for (uint32_t e = 0; e < 4; e++) w4[e] = out[4 * i + e];
        }
        *reinterpret_cast<uint4*>(st + 4 * i) = make_uint4(w4[0], w4[1], w4[2], w4[3]);
      }
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  constexpr uint32_t OB = kDstPacked ? C : 4;      // output bytes per pixel
#pragma unroll
  for (uint32_t p = 0; p < NP; p++) {
    const uint32_t q0 = (wave * np + p) * 64;
    if (!(p < np && q0 < nruns)) continue;
    const uint32_t words = min(64u, nruns - q0) * OW;
    const uint32_t chunks = words / 4;            // whole 16-byte chunks of this pass
    uint8_t* ob = v.dst + ((uint64_t)t0 * W + (uint64_t)q0 * KQ) * OB;
    const uint32_t* sp = lds + q0 * OW;
#pragma unroll
    for (uint32_t i = 0; i < (64 * OW / 4 + 63) / 64; i++) {
      const uint32_t ch = 64 * i + lane;
      if (ch < chunks) gstore4(ob + 16 * ch, *reinterpret_cast<const uint4*>(sp + 4 * ch));
    }
    if (lane < words % 4) ((gu32*)ob)[4 * chunks + lane] = sp[4 * chunks + lane];
  }
  return (carry ^ all) & 0xFFu;
}

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
