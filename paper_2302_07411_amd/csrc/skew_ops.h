// Device building blocks of the row-run round kernels (Sec. 2, Eq. (1)-(4),
// Algorithm 1's round loop), shared by the single-stream kernels
// (rounds_skew.hip) and the multi-stream batch kernel (batch.hip).
//
// Encryption (skew_tile): Eq. (1) sends source pixel (a, o) to row
// alpha = (a+o) mod H, column beta = (o + g(alpha)) mod W.  Seen from a block
// of destination rows [t0, t0+R), it is a column skew followed by one
// rotation per row: the tile T[k][o] (k = alpha - t0) holds source pixel
// ((t0+k-o) mod H, o), and row k of the result is row k of T rotated right by
// g(t0+k).  For a fixed source row a, the pixels that land in the tile are the
// R consecutive columns o = (t0+k-a) mod H (plus multiples of H when W > H),
// so the gather reads each source row as a contiguous run: one coalesced
// load instruction covers most of a run, and consecutive lanes write T[k][o]
// at LDS words that step by W+kRowPad+1, i.e. across banks.  The rotation is
// applied when the tile is read: row k starts at LDS word rowbase(k) =
// k*(W+kRowPad) + (g mod 4), so the four pixels at beta, beta+1, ... (beta a
// multiple of 4) sit at one 16-byte aligned address, and three copied words
// after each row cover reads that wrap past column W-1.
//
// Diffusion (Eq. 3) runs in chain order over bytes: each lane takes KQ
// consecutive pixels of a row (KQ*C bytes, KQ*C/4 words), packs the tile's
// pixel words into byte order with byte permutes, forms D = b ^ (Y + b) per
// byte, and XOR-prefixes the words (shift-XOR within a word, the previous
// word's last byte broadcast into the next).  Lane carries come from a DPP
// scan of lane totals inside the wavefront; wavefronts own consecutive
// stretches of runs, so one block scan of 16 wavefront totals per tile
// completes the chain.
//
// Decryption in one pass per tile (unskew_rows): X[a][o] = Y[alpha][beta]
// (Eq. 2) with Y Eq. (4) applied to the round input at (alpha, beta): seen
// from destination rows [t0, t0+R), source row alpha contributes R
// consecutive pixels beta (falling as the row rises), so the input pixels,
// their predecessors and their keystream bytes are read as contiguous runs.
#pragma once
#include "tile_ops.h"

namespace cv {
namespace skew {

using namespace tile;

constexpr uint32_t kThreads = 1024;
constexpr uint32_t kWaves = kThreads / 64;
constexpr uint32_t kRowPad = 8;      // per LDS row: 3 wrap words + up to 3 alignment words
constexpr uint32_t kMaxTilePix = 36 * kThreads;  // pixels of a tile: at most 36 per thread
// source rows in flight per thread in the gather (measured at 768x768x3: 8
// is fastest; 16 gains nothing, 24 spills registers)
constexpr uint32_t kGatherBatch = 8;


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


// ---------------------------------------------- one-pass decryption ---
// 12 bytes from a global address that is only 4-byte aligned.
typedef uint32_t v3u32a4 __attribute__((ext_vector_type(3), aligned(4)));
typedef __attribute__((address_space(1))) const v3u32a4 gcv3a4;
typedef uint32_t v2u32a4 __attribute__((ext_vector_type(2), aligned(4)));
typedef __attribute__((address_space(1))) const v2u32a4 gcv2a4;

// Input pixel x and its predecessor x-1 of a round input (packed or pixel
// words) with one load; x-1 is clamped to x at pixel 0 (the caller uses the
// seed there).  Returns the pixel word of x; *prev gets that of x-1.
template <uint32_t C, bool kSrcPacked>
__device__ __forceinline__ uint32_t pixel_pair(const View& v, uint32_t x, uint32_t* prev) {
  constexpr uint32_t msk = pixel_mask<C>();
  const uint32_t xp = x > 0 ? x - 1 : 0u;
  if constexpr (!kSrcPacked || C == 4) {
    const v2u32a4 w = *(gcv2a4*)(v.src + 4ull * xp);
    *prev = w.x;
    return x > 0 ? w.y : w.x;
  } else {
    // bytes [3xp, 3xp+6) lie in the 12 bytes from the dword holding byte
    // 3xp; near the end of the buffer the window starts 12 bytes before it
    const uint8_t* a = v.src + 3ull * xp;
    const uint8_t* al = (const uint8_t*)((uintptr_t)a & ~(uintptr_t)3);
    const uint8_t* win = al + 8 <= v.src_last ? al : v.src_last - 8;
    const v3u32a4 w = *(gcv3a4*)win;
    const uint32_t sh = (uint32_t)(a - win);  // 0..6
    const uint32_t p0 = sh >= 4 ? w.y : w.x, p1 = sh >= 4 ? w.z : w.y;
    *prev = __builtin_amdgcn_alignbyte(p1, p0, sh & 3u) & msk;
    const uint32_t s2 = sh + 3;               // 3..9
    const uint32_t c0 = s2 >= 8 ? w.z : (s2 >= 4 ? w.y : w.x);
    const uint32_t c1 = s2 >= 8 ? 0u : (s2 >= 4 ? w.z : w.y);
    const uint32_t cur = __builtin_amdgcn_alignbyte(c1, c0, s2 & 3u) & msk;
    return x > 0 ? cur : *prev;
  }
}

// The C keystream bytes of band-relative pixel p (one load).
template <uint32_t C>
__device__ __forceinline__ uint32_t ks_pixel(const uint8_t* kb, uint32_t p, const uint8_t* kb_last) {
  if constexpr (C == 4) return g32(kb)[p];
  const uint8_t* a = kb + 3ull * p;
  const uint8_t* al = (const uint8_t*)((uintptr_t)a & ~(uintptr_t)3);
  const uint8_t* win = al + 4 <= kb_last ? al : kb_last - 4;
  const v2u32a4 w = *(gcv2a4*)win;
  const uint32_t sh = (uint32_t)(a - win);  // 0..7
  const uint64_t x = ((uint64_t)w.y << 32) | w.x;
  return (uint32_t)(x >> (8 * sh)) & 0x00FFFFFFu;
}

// One pass of decryption round j for destination rows [t0, t0+R) into the
// LDS tile (row pitch W+4): thread (k, m) walks source rows alpha = s, s+A,
// ...; its pixel of row alpha is column o = (alpha - t0 - k) mod H (+ m*H),
// read at beta = (o + g(alpha)) mod W with its predecessor and keystream,
// and Eq. (4) gives the tile's T[k][o].  gsh: the frame's shift table in
// LDS; blo: first rows of the bands (n+1 entries); seed: the bands' seeds.
template <uint32_t C, bool kSrcPacked, bool kFull>
__device__ __forceinline__ void unskew_rows(const View& v, const Geom& g, uint32_t j, uint32_t t0,
                                            uint32_t R, const uint32_t* gsh, const uint32_t* blo,
                                            const uint32_t* seed, uint32_t* tile) {
  constexpr uint32_t kU = 4;
  constexpr uint32_t msk = pixel_mask<C>();
  const uint32_t W = g.W, H = g.H, pitch = W + 4;
  const uint32_t M = (W + H - 1) / H;
  const uint32_t per = R * M;
  const uint32_t A = kThreads / per;
  const uint32_t t = threadIdx.x;
  if (t >= per * A) return;
  const uint32_t k = t % R, rest = t / R, m = rest % M, s = rest / M;
  const uint32_t mH = m * H;
  uint32_t* row = tile + k * pitch;
  uint32_t b = 0;  // band of the current source row; rows only increase
  for (uint32_t al0 = s; al0 < H; al0 += kU * A) {
    uint32_t z[kU], zp[kU], kb[kU], o[kU], bb[kU];
    bool ok[kU], first[kU];
#pragma unroll
    for (uint32_t u = 0; u < kU; u++) {
      const uint32_t al = al0 + u * A;
      const uint32_t alc = al < H ? al : H - 1;
      while (blo[b + 1] <= alc) b++;
      const int32_t d = (int32_t)alc - (int32_t)(t0 + k);
      o[u] = (d < 0 ? (uint32_t)(d + (int32_t)H) : (uint32_t)d) + mH;
      ok[u] = al < H && (kFull || o[u] < W);
      const uint32_t oc = ok[u] ? o[u] : 0u;
      uint32_t beta = oc + gsh[alc];
      if (beta >= W) beta -= W;
      const uint32_t x = alc * W + beta;
      const uint32_t bs = blo[b] * W;  // the band's first pixel
      first[u] = x == bs;
      bb[u] = b;
      z[u] = pixel_pair<C, kSrcPacked>(v, x, &zp[u]);
      const uint64_t Sb = (uint64_t)(blo[b + 1] - blo[b]) * W * C;
      const uint8_t* kbase = v.ks + (uint64_t)g.r * bs * C + (uint64_t)j * Sb;
      kb[u] = ks_pixel<C>(kbase, x - bs, kbase + Sb - 4);
    }
#pragma unroll
    for (uint32_t u = 0; u < kU; u++) {
      const uint32_t pb = first[u] ? seed[bb[u]] : (zp[u] >> (8 * (C - 1))) & 0xFFu;
      const uint32_t zz = z[u] & msk, bk = kb[u] & msk;
      const uint32_t zs = ((zz << 8) | pb) & msk;
      if (ok[u]) row[o[u]] = sub_bytes(bk ^ zz ^ zs, bk) & msk;
    }
  }
}

}  // namespace skew
}  // namespace cv
