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
#include "cv_internal.h"

namespace cv {
namespace {

constexpr uint32_t kMaxThreads = 1024;
constexpr uint32_t kUnroll = 8;  // gather loads in flight per thread
constexpr uint32_t kPix = 16;    // pixels per thread in the diffusion pass (tile <= kPix*threads)

__device__ __forceinline__ uint32_t add_bytes(uint32_t a, uint32_t b) {
  return ((a & 0x7F7F7F7Fu) + (b & 0x7F7F7F7Fu)) ^ ((a ^ b) & 0x80808080u);
}

__device__ __forceinline__ uint32_t sub_bytes(uint32_t a, uint32_t b) {
  return ((a | 0x80808080u) - (b & 0x7F7F7F7Fu)) ^ ((a ^ ~b) & 0x80808080u);
}

template <uint32_t C>
__host__ __device__ constexpr uint32_t pixel_mask() {
  return C == 4 ? 0xFFFFFFFFu : 0x00FFFFFFu;
}

// Packed pixel `p` (C bytes at p*C) of a buffer whose last readable dword
// starts at `last`: two aligned dword loads and a byte funnel shift.  The
// second load is only needed when the pixel straddles; clamping it to `last`
// keeps it inside the buffer otherwise.
template <uint32_t C>
__device__ __forceinline__ uint32_t load_packed(const uint8_t* base, uint64_t p, const uint8_t* last) {
  if constexpr (C == 4) return reinterpret_cast<const uint32_t*>(base)[p];
  const uint8_t* a = base + p * 3;
  const uint8_t* al = reinterpret_cast<const uint8_t*>((uintptr_t)a & ~(uintptr_t)3);
  const uint32_t sh = (uint32_t)((uintptr_t)a & 3);
  const uint8_t* a1 = al + 4 <= last ? al + 4 : last;
  const uint32_t w0 = *reinterpret_cast<const uint32_t*>(al);
  const uint32_t w1 = *reinterpret_cast<const uint32_t*>(a1);
  return __builtin_amdgcn_alignbyte(w1, w0, sh) & 0x00FFFFFFu;
}

// Four packed pixels starting at a 16-byte-aligned group (12 or 16 bytes).
template <uint32_t C>
__device__ __forceinline__ uint4 load4_packed(const uint8_t* p) {
  if constexpr (C == 4) return *reinterpret_cast<const uint4*>(p);
  const uint32_t* w = reinterpret_cast<const uint32_t*>(p);
  const uint32_t k0 = w[0], k1 = w[1], k2 = w[2];
  return make_uint4(k0 & 0xFFFFFFu, (k0 >> 24) | ((k1 & 0xFFFFu) << 8),
                    (k1 >> 16) | ((k2 & 0xFFu) << 16), k2 >> 8);
}

template <uint32_t C>
__device__ __forceinline__ void store4_packed(uint8_t* p, uint4 v) {
  if constexpr (C == 4) {
    *reinterpret_cast<uint4*>(p) = v;
  } else {
    uint32_t* w = reinterpret_cast<uint32_t*>(p);
    w[0] = (v.x & 0xFFFFFFu) | (v.y << 24);
    w[1] = ((v.y >> 8) & 0xFFFFu) | (v.z << 16);
    w[2] = ((v.z >> 16) & 0xFFu) | (v.w << 8);
  }
}

// Exclusive XOR scan over the block in thread order; the XOR of all inputs
// comes back in `total`.
__device__ uint32_t block_xor_scan_excl(uint32_t v, uint32_t* sh, uint32_t& total) {
  const uint32_t lane = threadIdx.x & 63u, wid = threadIdx.x >> 6;
  const uint32_t nw = (blockDim.x + 63u) >> 6;
  uint32_t inc = v;
#pragma unroll
  for (uint32_t d = 1; d < 64; d <<= 1) {
    const uint32_t t = __shfl_up(inc, d, 64);
    if (lane >= d) inc ^= t;
  }
  if (lane == 63) sh[wid] = inc;
  __syncthreads();
  uint32_t before = 0, all = 0;
  for (uint32_t w = 0; w < nw; w++) {
    const uint32_t s = sh[w];
    if (w < wid) before ^= s;
    all ^= s;
  }
  __syncthreads();
  total = all;
  return before ^ inc ^ v;
}

// Frame views of one round: source and destination, packed or pixel words.
struct View {
  const uint8_t* src;       // frame base
  uint8_t* dst;             // frame base
  const uint8_t* src_last;  // last readable dword of the source buffer
  const uint8_t* ks;        // frame's keystream base (packed, canonical layout)
  const uint32_t* gm;       // frame's g(alpha) mod W
};

template <uint32_t C, bool kSrcPacked>
__device__ __forceinline__ uint32_t src_pixel(const View& v, uint64_t p) {
  if constexpr (kSrcPacked) return load_packed<C>(v.src, p, v.src_last);
  return reinterpret_cast<const uint32_t*>(v.src)[p];
}

// Gather of Eq. (1) for destination rows [t0, t0+R): tile[k*W + beta] =
// source pixel (a, o) with alpha = t0+k = (a+o) mod H, beta = (o+g) mod W.
// Thread = (k, slot): consecutive lanes take consecutive k, i.e. consecutive
// pixels of one source row's run; each thread walks source rows a = slot,
// slot+ns, ... with incremental index arithmetic, kUnroll loads in flight.
template <uint32_t C, bool kSrcPacked>
__device__ __forceinline__ void gather_rows(const View& v, const Geom& g, uint32_t t0, uint32_t R,
                                            uint32_t* tile) {
  const uint32_t tid = threadIdx.x, T = blockDim.x;
  const uint32_t W = g.W, H = g.H;
  const uint32_t M = (W + H - 1) / H;   // runs per source row
  const uint32_t ns = (T / R) / M * M;  // slots in use, a multiple of M
  const uint32_t k = tid % R, slot = tid / R;
  if (slot >= ns) return;
  const uint32_t alpha = t0 + k;
  const uint32_t shift = v.gm[alpha];
  uint32_t* drow = tile + (size_t)k * W;
  const uint32_t m = slot % M, astep = ns / M;
  const uint32_t dstep = astep % H;     // decrease of (alpha - a) mod H per step
  uint32_t a = slot / M;
  uint32_t ob = alpha + H - a % H;      // (alpha - a) mod H
  if (ob >= H) ob -= H;
  while (a < H) {
    uint32_t val[kUnroll], beta[kUnroll];
    bool ok[kUnroll];
#pragma unroll
    for (uint32_t u = 0; u < kUnroll; u++) {
      const uint32_t o = ob + m * H;
      ok[u] = a < H && o < W;
      const uint32_t oc = ok[u] ? o : 0;
      const uint32_t bs = oc + shift;
      beta[u] = bs >= W ? bs - W : bs;
      val[u] = src_pixel<C, kSrcPacked>(v, ok[u] ? a * W + oc : 0u);
      a += astep;
      ob = ob >= dstep ? ob - dstep : ob + H - dstep;
    }
#pragma unroll
    for (uint32_t u = 0; u < kUnroll; u++)
      if (ok[u]) drow[beta[u]] = val[u];
  }
}

// Encryption of rows [t0, t0+R) of band [lo, hi), round j: gather (Eq. 1)
// into the LDS tile, then diffusion (Eq. 3) seeded with `carry` in one pass
// over registers -- every thread owns kPix consecutive pixels of the chain:
// D = b ^ (Y + b), XOR-reduce, block scan for its carry, prefix, store.
// Returns the carry into the next tile of the band.
template <uint32_t C, bool kSrcPacked, bool kDstPacked>
__device__ uint32_t enc_tile(const View& v, const Geom& g, uint32_t j, uint32_t lo, uint32_t hi,
                             uint32_t t0, uint32_t R, uint32_t carry, uint32_t* tile,
                             uint32_t* scan_sh) {
  const uint32_t tid = threadIdx.x;
  const uint32_t W = g.W;
  const uint32_t npix = R * W;
  const uint64_t S = (uint64_t)(hi - lo) * W * C;
  const uint8_t* kt = v.ks + (uint64_t)g.r * lo * W * C + (uint64_t)j * S + (uint64_t)(t0 - lo) * W * C;
  const uint32_t p0 = tid * kPix;
  const bool mine = p0 < npix;  // npix is a multiple of kPix
  // keystream of this thread's pixels first: its latency hides behind the gather
  uint4 b[kPix / 4];
#pragma unroll
  for (uint32_t i = 0; i < kPix / 4; i++)
    b[i] = mine ? load4_packed<C>(kt + (uint64_t)(p0 + 4 * i) * C) : make_uint4(0, 0, 0, 0);
  gather_rows<C, kSrcPacked>(v, g, t0, R, tile);
  __syncthreads();
  constexpr uint32_t msk = pixel_mask<C>();
  uint32_t d[kPix];
  uint32_t red = 0;
#pragma unroll
  for (uint32_t i = 0; i < kPix / 4; i++) {
    const uint4 y = mine ? reinterpret_cast<const uint4*>(tile)[p0 / 4 + i] : make_uint4(0, 0, 0, 0);
    d[4 * i + 0] = (b[i].x ^ add_bytes(y.x, b[i].x)) & msk;
    d[4 * i + 1] = (b[i].y ^ add_bytes(y.y, b[i].y)) & msk;
    d[4 * i + 2] = (b[i].z ^ add_bytes(y.z, b[i].z)) & msk;
    d[4 * i + 3] = (b[i].w ^ add_bytes(y.w, b[i].w)) & msk;
    red ^= d[4 * i] ^ d[4 * i + 1] ^ d[4 * i + 2] ^ d[4 * i + 3];
  }
  red ^= red >> 16;
  red ^= red >> 8;
  uint32_t total;
  const uint32_t excl = block_xor_scan_excl(red & 0xFFu, scan_sh, total);
  uint32_t c = (carry ^ excl) & 0xFFu;
#pragma unroll
  for (uint32_t i = 0; i < kPix; i++) {
    uint32_t z = d[i];
    z ^= z << 8;
    z ^= z << 16;
    z ^= c * 0x01010101u;
    c = z >> 24;
    d[i] = z & msk;
  }
  if (mine) {
    if constexpr (kDstPacked) {
      uint8_t* o = v.dst + ((uint64_t)t0 * W + p0) * C;
#pragma unroll
      for (uint32_t i = 0; i < kPix / 4; i++)
        store4_packed<C>(o + 4 * i * C, make_uint4(d[4 * i], d[4 * i + 1], d[4 * i + 2], d[4 * i + 3]));
    } else {
      uint4* o = reinterpret_cast<uint4*>(v.dst + ((uint64_t)t0 * W + p0) * 4);
#pragma unroll
      for (uint32_t i = 0; i < kPix / 4; i++)
        o[i] = make_uint4(d[4 * i], d[4 * i + 1], d[4 * i + 2], d[4 * i + 3]);
    }
  }
  return (carry ^ total) & 0xFFu;
}

// Seed of band `band` for round j of encryption: the last byte of band
// (band+1) mod n after confusion, before diffusion, read from the round
// input through the inverse of Eq. (1).
template <uint32_t C, bool kSrcPacked>
__device__ uint32_t enc_seed(const View& v, const Geom& g, uint32_t band) {
  const uint32_t nb = band + 1 == g.n ? 0 : band + 1;
  const uint32_t alpha = (uint32_t)band_lo(g.H, g.n, nb + 1) - 1;
  uint32_t o = (g.W - 1) + g.W - v.gm[alpha];
  if (o >= g.W) o -= g.W;
  uint32_t a = alpha + g.H - (o % g.H);
  if (a >= g.H) a -= g.H;
  return (src_pixel<C, kSrcPacked>(v, (uint64_t)a * g.W + o) >> (8 * (C - 1))) & 0xFFu;
}

// Decryption of rows [t0, t0+R) of the frame, round j: every output pixel
// (a, o) is the confused pixel (alpha, beta) of Eq. (1) with its diffusion
// undone by Eq. (4) as it is read.
template <uint32_t C, bool kSrcPacked, bool kDstPacked>
__device__ void dec_tile(const View& v, const Geom& g, uint32_t j, uint32_t t0, uint32_t R,
                         uint32_t* tile, const uint32_t* blo, const uint32_t* seed) {
  const uint32_t tid = threadIdx.x, T = blockDim.x;
  const uint32_t W = g.W, H = g.H;
  constexpr uint32_t msk = pixel_mask<C>();
  {
    const uint32_t M = (W + H - 1) / H;
    const uint32_t ns = (T / R) / M * M;
    const uint32_t k = tid % R, slot = tid / R;
    if (slot < ns) {
      const uint32_t a = t0 + k;
      uint32_t* drow = tile + (size_t)k * W;
      const uint32_t m = slot % M, astep = ns / M;
      constexpr uint32_t kU = kUnroll / 2;
      uint32_t bi = 0;  // band of the current row; rows only increase
      for (uint32_t alpha0 = slot / M; alpha0 < H; alpha0 += kU * astep) {
        uint32_t zv[kU], pv[kU], bv[kU], ov[kU], sv[kU];
        bool ok[kU], first[kU];
#pragma unroll
        for (uint32_t u = 0; u < kU; u++) {
          const uint32_t al = alpha0 + u * astep;
          ok[u] = al < H;
          const uint32_t alpha = ok[u] ? al : H - 1;
          while (blo[bi + 1] <= alpha) bi++;
          const uint64_t band_pix = (uint64_t)blo[bi] * W;  // first pixel of the band
          const uint64_t Sb = (uint64_t)(blo[bi + 1] - blo[bi]) * W * C;
          const uint8_t* kb = v.ks + (uint64_t)g.r * band_pix * C + (uint64_t)j * Sb;
          uint32_t ob = alpha + H - a;
          if (ob >= H) ob -= H;
          const uint32_t o = ob + m * H;
          ok[u] = ok[u] && o < W;
          const uint32_t oc = ok[u] ? o : 0;
          const uint32_t shift = v.gm[alpha];
          const uint32_t beta = oc + shift >= W ? oc + shift - W : oc + shift;
          const uint64_t x = (uint64_t)alpha * W + beta;  // flat pixel
          first[u] = x == band_pix;
          ov[u] = oc;
          sv[u] = seed[bi];
          zv[u] = src_pixel<C, kSrcPacked>(v, x);
          pv[u] = src_pixel<C, kSrcPacked>(v, first[u] ? x : x - 1);
          bv[u] = load_packed<C>(kb, x - band_pix, kb + Sb - 4);
        }
#pragma unroll
        for (uint32_t u = 0; u < kU; u++) {
          if (!ok[u]) continue;
          const uint32_t prev = first[u] ? sv[u] : (pv[u] >> (8 * (C - 1))) & 0xFFu;
          const uint32_t b = bv[u] & msk, z = zv[u];
          const uint32_t zp = ((z << 8) | prev) & msk;
          drow[ov[u]] = sub_bytes(b ^ z ^ zp, b) & msk;
        }
      }
    }
  }
  __syncthreads();
  const uint32_t npix = R * W;
  if constexpr (kDstPacked) {
    uint8_t* d = v.dst + (uint64_t)t0 * W * C;
    for (uint32_t q = tid; q < npix / 4; q += T)
      store4_packed<C>(d + (uint64_t)q * 4 * C, reinterpret_cast<const uint4*>(tile)[q]);
  } else {
    uint4* d = reinterpret_cast<uint4*>(v.dst + (uint64_t)t0 * W * 4);
    for (uint32_t q = tid; q < npix / 4; q += T) d[q] = reinterpret_cast<const uint4*>(tile)[q];
  }
  __syncthreads();
}

// Per-band first rows and recovered decryption seeds of round j: the seed of
// band i is the pre-diffusion last byte of band (i+1) mod n, i.e. Eq. (4) on
// that band's last two cipher bytes.
template <uint32_t C, bool kSrcPacked>
__device__ void dec_seeds(const View& v, const Geom& g, uint32_t j, uint32_t* blo, uint32_t* seed) {
  for (uint32_t i = threadIdx.x; i <= g.n; i += blockDim.x) blo[i] = (uint32_t)band_lo(g.H, g.n, i);
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < g.n; i += blockDim.x) {
    const uint32_t ip = i + 1 == g.n ? 0 : i + 1;
    const uint64_t first = (uint64_t)blo[ip] * g.W, end = (uint64_t)blo[ip + 1] * g.W;
    const uint64_t Sp = (end - first) * C;
    const uint8_t bp = v.ks[(uint64_t)g.r * first * C + (uint64_t)j * Sp + Sp - 1];
    const uint32_t zl = src_pixel<C, kSrcPacked>(v, end - 1);  // last pixel of band ip
    const uint8_t z1 = (uint8_t)(zl >> (8 * (C - 1))), z0 = (uint8_t)(zl >> (8 * (C - 2)));
    seed[i] = (uint8_t)((bp ^ z1 ^ z0) - bp);
  }
  __syncthreads();
}

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

__device__ __forceinline__ uint32_t xcc_id() {
  uint32_t v;
  asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID)" : "=s"(v));
  return v & 0xFu;
}

// Record this workgroup's XCC for its group; a different XCC than the one a
// group member recorded first raises `err`.
__device__ __forceinline__ void check_group_xcc(uint32_t* slot, uint32_t* err) {
  if (threadIdx.x == 0) {
    const uint32_t mine = xcc_id();
    uint32_t expect = 0xFFFFFFFFu;
    if (!__hip_atomic_compare_exchange_strong(slot, &expect, mine, __ATOMIC_RELAXED,
                                              __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) &&
        expect != mine)
      __hip_atomic_store(err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

__device__ __forceinline__ bool group_barrier(uint32_t* ctr, uint32_t target, uint32_t spin_limit,
                                              uint32_t* err) {
  __shared__ uint32_t ok_sh;
  // release: this wavefront's global stores have reached the XCD's L2
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_waitcnt(0);
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __syncthreads();
  if (threadIdx.x == 0) {
    __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    uint32_t spins = 0, ok = 1;
    while ((int32_t)(__hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) - target) < 0) {
      if (++spins > spin_limit || __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
        __hip_atomic_store(err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        ok = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) ok = 0;
    // acquire: invalidate the CU's L1 (and clean L2 lines) before any
    // wavefront of the workgroup reads what the other members wrote
    asm volatile("buffer_inv sc1\n\ts_waitcnt vmcnt(0)" ::: "memory");
    ok_sh = ok;
  }
  __syncthreads();
  return ok_sh != 0;
}

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
