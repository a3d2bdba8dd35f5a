// Device building blocks of the pixel-word round kernels (Sec. 2, Eq. (1)-(4),
// Algorithm 2), shared by the single-stream kernels (rounds_pw.hip) and the
// multi-stream batch kernel (batch.hip).  See rounds_pw.hip for the layout.
#pragma once
#include "cv_internal.h"

namespace cv {
namespace tile {


constexpr uint32_t kMaxThreads = 1024;

// Global-memory views.  Frame, keystream and scratch pointers reach the
// kernels through argument structs, where the compiler cannot see that they
// point to global memory; without these casts it emits flat accesses, which
// also count against the LDS wait counter and serialise the gathers.
typedef __attribute__((address_space(1))) const uint32_t gcu32;
typedef __attribute__((address_space(1))) uint32_t gu32;
typedef __attribute__((address_space(1))) const uint8_t gcu8;
typedef unsigned int v4u32 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(1))) v4u32 gv4;
__device__ __forceinline__ const gcu32* g32(const void* p) { return (const gcu32*)p; }
__device__ __forceinline__ uint4 gload4(const void* p) {
  const v4u32 x = *(const gv4*)p;
  return make_uint4(x.x, x.y, x.z, x.w);
}
// 16 bytes from a global address that is only 4-byte aligned: one
// global_load_dwordx4 instead of four dword loads.
typedef uint32_t v4u32a4 __attribute__((ext_vector_type(4), aligned(4)));
typedef __attribute__((address_space(1))) const v4u32a4 gcv4a4;
__device__ __forceinline__ v4u32a4 gload4u(const void* p) { return *(gcv4a4*)p; }

__device__ __forceinline__ void gstore4(void* p, uint4 v) {
  v4u32 x;
  x.x = v.x;
  x.y = v.y;
  x.z = v.z;
  x.w = v.w;
  *(gv4*)p = x;
}
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
  if constexpr (C == 4) return g32(base)[p];
  const uint8_t* a = base + p * 3;
  const uint8_t* al = reinterpret_cast<const uint8_t*>((uintptr_t)a & ~(uintptr_t)3);
  const uint32_t sh = (uint32_t)((uintptr_t)a & 3);
  const uint8_t* a1 = al + 4 <= last ? al + 4 : last;
  const uint32_t w0 = *g32(al);
  const uint32_t w1 = *g32(a1);
  return __builtin_amdgcn_alignbyte(w1, w0, sh) & 0x00FFFFFFu;
}

// Four packed pixels starting at a 16-byte-aligned group (12 or 16 bytes).
template <uint32_t C>
__device__ __forceinline__ uint4 load4_packed(const uint8_t* p) {
  if constexpr (C == 4) return gload4(p);
  const gcu32* w = g32(p);
  const uint32_t k0 = w[0], k1 = w[1], k2 = w[2];
  return make_uint4(k0 & 0xFFFFFFu, (k0 >> 24) | ((k1 & 0xFFFFu) << 8),
                    (k1 >> 16) | ((k2 & 0xFFu) << 16), k2 >> 8);
}

template <uint32_t C>
__device__ __forceinline__ void store4_packed(uint8_t* p, uint4 v) {
  if constexpr (C == 4) {
    gstore4(p, v);
  } else {
    gu32* w = (gu32*)p;
    w[0] = (v.x & 0xFFFFFFu) | (v.y << 24);
    w[1] = ((v.y >> 8) & 0xFFFFu) | (v.z << 16);
    w[2] = ((v.z >> 16) & 0xFFu) | (v.w << 8);
  }
}

// Byte order <-> pixel words for 4 pixels (C = 3): 3 packed words hold the
// 12 bytes of 4 pixel words.
__device__ __forceinline__ void pack4(const uint32_t* w, uint32_t* P) {
  P[0] = __builtin_amdgcn_perm(w[1], w[0], 0x04020100u);
  P[1] = __builtin_amdgcn_perm(w[2], w[1], 0x05040201u);
  P[2] = __builtin_amdgcn_perm(w[3], w[2], 0x06050402u);
}

__device__ __forceinline__ void unpack4(const uint32_t* P, uint32_t* w) {
  w[0] = __builtin_amdgcn_perm(P[1], P[0], 0x0C020100u);
  w[1] = __builtin_amdgcn_perm(P[1], P[0], 0x0C050403u);
  w[2] = __builtin_amdgcn_perm(P[2], P[1], 0x0C040302u);
  w[3] = __builtin_amdgcn_perm(P[2], P[2], 0x0C030201u);
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
  return g32(v.src)[p];
}

// Gather of Eq. (1) for destination rows [t0, t0+R): tile[k*W + beta] =
// source pixel (a, o) with alpha = t0+k = (a+o) mod H, beta = (o+g) mod W.
// Thread = (k, slot): consecutive lanes take consecutive k, i.e. consecutive
// pixels of one source row's run; each thread walks source rows a = slot,
// slot+ns, ... with incremental index arithmetic.  Loads go out kUnroll at a
// time and the next batch is issued before the current one is stored; the
// stores are unconditional (a lane past the frame writes to `sink`).
template <uint32_t C, bool kSrcPacked>
__device__ __forceinline__ void gather_rows(const View& v, const Geom& g, uint32_t t0, uint32_t R,
                                            uint32_t* tile) {
  __shared__ uint32_t sink;
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
  uint32_t val[kUnroll];
  uint32_t* dst[kUnroll];
  auto issue = [&](uint32_t* vv, uint32_t** dd) {
#pragma unroll
    for (uint32_t u = 0; u < kUnroll; u++) {
      const uint32_t o = ob + m * H;
      const bool ok = a < H && o < W;
      const uint32_t oc = ok ? o : 0;
      const uint32_t bs = oc + shift;
      dd[u] = ok ? drow + (bs >= W ? bs - W : bs) : &sink;
      vv[u] = src_pixel<C, kSrcPacked>(v, ok ? a * W + oc : 0u);
      a += astep;
      ob = ob >= dstep ? ob - dstep : ob + H - dstep;
    }
  };
  issue(val, dst);
  while (a < H) {
    uint32_t val2[kUnroll];
    uint32_t* dst2[kUnroll];
    issue(val2, dst2);
#pragma unroll
    for (uint32_t u = 0; u < kUnroll; u++) *dst[u] = val[u];
#pragma unroll
    for (uint32_t u = 0; u < kUnroll; u++) {
      val[u] = val2[u];
      dst[u] = dst2[u];
    }
  }
#pragma unroll
  for (uint32_t u = 0; u < kUnroll; u++) *dst[u] = val[u];
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
  // keystream of this thread's pixels first: its latency hides behind the
  // gather.  With C = 3 the thread's 3*kPix bytes come in 16-byte loads (a
  // dword load instruction at this lane stride touches 24 cache lines).
  uint4 b[kPix / 4];
  if constexpr (C == 3) {
    uint32_t kw[kPix * 3 / 4];
    const uint8_t* kp = kt + (uint64_t)(mine ? p0 : 0u) * 3;
#pragma unroll
    for (uint32_t i = 0; i < kPix * 3 / 16; i++) {
      const v4u32a4 w = gload4u(kp + 16 * i);
      kw[4 * i] = w.x;
      kw[4 * i + 1] = w.y;
      kw[4 * i + 2] = w.z;
      kw[4 * i + 3] = w.w;
    }
#pragma unroll
    for (uint32_t i = 0; i < kPix / 4; i++) {
      const uint32_t k0 = kw[3 * i], k1 = kw[3 * i + 1], k2 = kw[3 * i + 2];
      b[i] = mine ? make_uint4(k0 & 0xFFFFFFu, (k0 >> 24) | ((k1 & 0xFFFFu) << 8),
                               (k1 >> 16) | ((k2 & 0xFFu) << 16), k2 >> 8)
                  : make_uint4(0, 0, 0, 0);
    }
  } else {
#pragma unroll
    for (uint32_t i = 0; i < kPix / 4; i++)
      b[i] = mine ? load4_packed<C>(kt + (uint64_t)(p0 + 4 * i) * C) : make_uint4(0, 0, 0, 0);
  }
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
  // Stores staged through the thread's own tile words (it alone read them),
  // so that each store instruction of a wavefront writes 1 KB of
  // consecutive bytes: packed (C = 3) a thread's 16 pixels are 12 words.
  constexpr uint32_t OW = kDstPacked && C == 3 ? kPix * 3 / 4 : kPix;  // output words per thread
  if (mine) {
#pragma unroll
    for (uint32_t i = 0; i < kPix / 4; i++) {
      if constexpr (OW == kPix) {
        reinterpret_cast<uint4*>(tile)[p0 / 4 + i] = make_uint4(d[4 * i], d[4 * i + 1], d[4 * i + 2], d[4 * i + 3]);
      } else {
        uint32_t* w = tile + p0 + 3 * i;
        w[0] = (d[4 * i] & 0xFFFFFFu) | (d[4 * i + 1] << 24);
        w[1] = ((d[4 * i + 1] >> 8) & 0xFFFFu) | (d[4 * i + 2] << 16);
        w[2] = ((d[4 * i + 2] >> 16) & 0xFFu) | (d[4 * i + 3] << 8);
      }
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  {
    const uint32_t lane = tid & 63u, pw = (tid - lane) * kPix;  // the wavefront's first pixel
    if (pw < npix) {
      const uint32_t threads = min(64u, (npix - pw) / kPix);    // threads of the wavefront with pixels
      const uint32_t chunks = threads * OW / 4;                 // 16-byte chunks (OW % 4 == 0)
      uint8_t* o = v.dst + ((uint64_t)t0 * W + pw) * (kDstPacked ? C : 4);
#pragma unroll
      for (uint32_t i = 0; i < OW / 4; i++) {
        const uint32_t c = 64 * i + lane;  // chunk c: thread c / (OW/4), its words 4*(c % (OW/4))
        if (c < chunks) {
          const uint32_t th = c / (OW / 4), wd = 4 * (c % (OW / 4));
          gstore4(o + 16 * c, *reinterpret_cast<const uint4*>(tile + pw + th * kPix + wd));
        }
      }
    }
  }
  return (carry ^ total) & 0xFFu;
}

// Seed of band `band` for round j of encryption: the last byte of band
// (band+1) mod n after confusion, before diffusion, read from the round
// input through the inverse of Eq. (1).  enc_seed_index gives the source
// pixel index of that byte (it depends on the frame's shift table only).
__device__ __forceinline__ uint64_t enc_seed_index(const View& v, const Geom& g, uint32_t band) {
  const uint32_t nb = band + 1 == g.n ? 0 : band + 1;
  const uint32_t alpha = (uint32_t)band_lo(g.H, g.n, nb + 1) - 1;
  uint32_t o = (g.W - 1) + g.W - v.gm[alpha];
  if (o >= g.W) o -= g.W;
  uint32_t a = alpha + g.H - (o % g.H);
  if (a >= g.H) a -= g.H;
  return (uint64_t)a * g.W + o;
}

template <uint32_t C, bool kSrcPacked>
__device__ uint32_t enc_seed(const View& v, const Geom& g, uint32_t band) {
  return (src_pixel<C, kSrcPacked>(v, enc_seed_index(v, g, band)) >> (8 * (C - 1))) & 0xFFu;
}

// Decryption of rows [t0, t0+R) of the frame, round j: every output pixel
// (a, o) is the confused pixel (alpha, beta) of Eq. (1) with its diffusion
// undone by Eq. (4) as it is read.
template <uint32_t C, bool kSrcPacked, bool kDstPacked>
__device__ void dec_tile(const View& v, const Geom& g, uint32_t j, uint32_t t0, uint32_t R,
                         uint32_t* tile, const uint32_t* blo, const uint32_t* seed) {
  __shared__ uint32_t sink;  // target of the stores of lanes past the frame
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
          const uint32_t prev = first[u] ? sv[u] : (pv[u] >> (8 * (C - 1))) & 0xFFu;
          const uint32_t b = bv[u] & msk, z = zv[u];
          const uint32_t zp = ((z << 8) | prev) & msk;
          *(ok[u] ? drow + ov[u] : &sink) = sub_bytes(b ^ z ^ zp, b) & msk;
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
    uint8_t* d = v.dst + (uint64_t)t0 * W * 4;
    for (uint32_t q = tid; q < npix / 4; q += T) gstore4(d + 16 * (uint64_t)q, reinterpret_cast<const uint4*>(tile)[q]);
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
    const uint8_t bp = ((const gcu8*)v.ks)[(uint64_t)g.r * first * C + (uint64_t)j * Sp + Sp - 1];
    const uint32_t zl = src_pixel<C, kSrcPacked>(v, end - 1);  // last pixel of band ip
    const uint8_t z1 = (uint8_t)(zl >> (8 * (C - 1))), z0 = (uint8_t)(zl >> (8 * (C - 2)));
    seed[i] = (uint8_t)((bp ^ z1 ^ z0) - bp);
  }
  __syncthreads();
}


// ------------------------------------------------ frame-group barrier ---
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

// Group barrier in two halves, so that work independent of the other
// members (loads of the next round's keystream) can be issued in between.
// Arrive: this wavefront's global stores have reached the XCD's L2
// (release), then one atomic increment per workgroup.
__device__ __forceinline__ void group_arrive(uint32_t* ctr) {
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_waitcnt(0);
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __syncthreads();
  if (threadIdx.x == 0) __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Wait until the counter reaches `target` (bounded: gives up after
// spin_limit polls or when another member raised `err`, raising it too),
// then acquire: invalidate the CU's L1 before any wavefront of the workgroup
// reads what the other members wrote.  False if the barrier failed.
__device__ __forceinline__ bool group_wait(uint32_t* ctr, uint32_t target, uint32_t spin_limit,
                                           uint32_t* err) {
  __shared__ uint32_t ok_sh;
  if (threadIdx.x == 0) {
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
    asm volatile("buffer_inv sc1\n\ts_waitcnt vmcnt(0)" ::: "memory");
    ok_sh = ok;
  }
  __syncthreads();
  return ok_sh != 0;
}

__device__ __forceinline__ bool group_barrier(uint32_t* ctr, uint32_t target, uint32_t spin_limit,
                                              uint32_t* err) {
  group_arrive(ctr);
  return group_wait(ctr, target, spin_limit, err);
}

}  // namespace tile
}  // namespace cv
