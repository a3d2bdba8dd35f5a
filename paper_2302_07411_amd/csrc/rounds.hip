// One confusion+diffusion round and its inverse, for gfx950 (Sec. 2,
// Eq. (1)-(4), Algorithm 2).
//
// Confusion (Eq. 1) sends pixel (a,o) to (alpha,beta) = ((a+o) mod H,
// (o+g[alpha]) mod W).  Seen from a block of destination rows
// [t0,t0+R), source row a contributes the pixels with o = (t0+k-a) mod H
// (+ multiples of H while o < W), k = 0..R-1: a contiguous run of R pixels
// per source row, wrapping at most once.  The gather is therefore driven by
// source rows: consecutive lanes take consecutive k, so a wavefront reads a
// few short contiguous runs, and writes each pixel into the LDS tile at its
// destination (k, beta).
//
// Diffusion (Eq. 3), C_k = b_k ^ ((P_k + b_k) mod 256) ^ C_{k-1}, unrolls to
// C_k = s_d ^ D_0 ^ ... ^ D_k with D_k = b_k ^ ((P_k + b_k) mod 256): XOR is
// associative, so the band's chain is an inclusive XOR scan seeded with s_d.
// The tile is scanned in LDS: D is formed 4 bytes at a time (SWAR byte-wise
// add), every thread reduces a contiguous segment, a block-wide exclusive
// scan gives each segment its carry, and each segment is re-scanned with it.
// A band larger than one tile is walked tile by tile, carrying the last byte.
//
// The seed s_d of band i is the last byte of band (i+1) mod n after
// confusion and before diffusion (the only reading under which all bands
// can diffuse concurrently); it is read straight from the round input
// through the inverse of Eq. (1).
//
// Inverse diffusion (Eq. 4), P_k = (b_k ^ C_k ^ C_{k-1}) - b_k, is
// element-wise, so decryption needs no scan: the inverse round gathers
// (Eq. 2) and undoes the diffusion of each byte as it reads it.
#include "cv_internal.h"

namespace cv {
namespace {

constexpr uint32_t kMaxThreads = 1024;

// Byte-wise (mod 256) addition of four packed bytes.
__device__ __forceinline__ uint32_t add_bytes(uint32_t a, uint32_t b) {
  return ((a & 0x7F7F7F7Fu) + (b & 0x7F7F7F7Fu)) ^ ((a ^ b) & 0x80808080u);
}

// Load bytes [p, p+len) (len <= 4) as a little-endian word; bytes past len
// are zero.  Reads only inside [p, p+len).
__device__ __forceinline__ uint32_t load_bytes(const uint8_t* p, uint32_t len) {
  if (len >= 4 && (((uintptr_t)p) & 3u) == 0) return *reinterpret_cast<const uint32_t*>(p);
  uint32_t v = 0;
  for (uint32_t i = 0; i < len && i < 4; i++) v |= (uint32_t)p[i] << (8 * i);
  return v;
}

__device__ __forceinline__ void store_bytes(uint8_t* p, uint32_t v, uint32_t len) {
  if (len >= 4 && (((uintptr_t)p) & 3u) == 0) {
    *reinterpret_cast<uint32_t*>(p) = v;
    return;
  }
  for (uint32_t i = 0; i < len && i < 4; i++) p[i] = (uint8_t)(v >> (8 * i));
}

// Exclusive XOR scan over the block in thread order; `total` gets the XOR
// of all inputs.  `sh` holds one word per wavefront.
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

// Pixel index pieces of the inverse of Eq. (1) for destination (alpha,beta).
__device__ __forceinline__ uint64_t source_byte(uint32_t alpha, uint32_t beta, const Geom& g,
                                                const uint32_t* gm) {
  uint32_t o = beta + g.W - gm[alpha];
  if (o >= g.W) o -= g.W;
  uint32_t a = alpha + g.H - (o % g.H);
  if (a >= g.H) a -= g.H;
  return ((uint64_t)a * g.W + o) * g.C;
}

// ------------------------------------------------------------ encrypt ----
__global__ __launch_bounds__(kMaxThreads) void round_enc_kernel(RoundArgs A) {
  extern __shared__ __align__(16) uint8_t lds[];
  __shared__ uint32_t scan_sh[kMaxThreads / 64];
  __shared__ uint32_t carry_sh;
  const Geom g = A.g;
  const uint32_t band = blockIdx.x, frame = blockIdx.y;
  const uint32_t tid = threadIdx.x, T = blockDim.x;
  const uint64_t row = (uint64_t)g.W * g.C;
  const uint8_t* src = A.src + (uint64_t)frame * A.frame_bytes;
  uint8_t* dst = A.dst + (uint64_t)frame * A.frame_bytes;
  const uint32_t* gm = A.gm + (uint64_t)frame * g.H;
  const uint32_t lo = (uint32_t)band_lo(g.H, g.n, band), hi = (uint32_t)band_lo(g.H, g.n, band + 1);
  const uint64_t S = (uint64_t)(hi - lo) * row;
  const uint8_t* ks = A.ks + (uint64_t)frame * A.ks_stride + (uint64_t)g.r * lo * row +
                      (uint64_t)A.j * S;

  if (tid == 0) {
    // s_d: last byte of band (band+1) mod n after confusion, before diffusion
    const uint32_t nb = band + 1 == g.n ? 0 : band + 1;
    const uint32_t alpha = (uint32_t)band_lo(g.H, g.n, nb + 1) - 1;
    carry_sh = src[source_byte(alpha, g.W - 1, g, gm) + g.C - 1];
  }

  const uint32_t M = (g.W + g.H - 1) / g.H;  // runs per source row
  for (uint32_t t0 = lo; t0 < hi; t0 += A.tile_rows) {
    const uint32_t R = min(A.tile_rows, hi - t0);
    const uint32_t St = R * (uint32_t)row;

    // ---- gather (Eq. 1): thread = (k, slot); slot walks source rows ----
    const uint32_t nslots = T / R;
    const uint32_t k = tid % R, slot = tid / R;
    if (slot < nslots) {
      const uint32_t alpha = t0 + k;
      const uint32_t shift = gm[alpha];
      uint8_t* drow = lds + (uint64_t)k * row;
      for (uint32_t a = slot; a < g.H; a += nslots) {
        uint32_t ob = alpha + g.H - a;
        if (ob >= g.H) ob -= g.H;
        for (uint32_t m = 0; m < M; m++) {
          const uint32_t o = ob + m * g.H;
          if (o >= g.W) break;
          uint32_t beta = o + shift;
          if (beta >= g.W) beta -= g.W;
          const uint8_t* sp = src + ((uint64_t)a * g.W + o) * g.C;
          uint8_t* dp = drow + (uint64_t)beta * g.C;
          for (uint32_t c = 0; c < g.C; c++) dp[c] = sp[c];
        }
      }
    }
    __syncthreads();

    // ---- D = b ^ (Y + b) in place, 4 bytes per thread-step (coalesced) ----
    const uint32_t nwords = (St + 3) / 4;
    const uint8_t* kt = ks + (uint64_t)(t0 - lo) * row;
    uint32_t* lw = reinterpret_cast<uint32_t*>(lds);
    for (uint32_t w = tid; w < nwords; w += T) {
      const uint32_t len = min(4u, St - 4 * w);
      const uint32_t b = load_bytes(kt + 4 * w, len);
      const uint32_t mask = len >= 4 ? 0xFFFFFFFFu : ((1u << (8 * len)) - 1u);
      lw[w] = (b ^ add_bytes(lw[w], b)) & mask;
    }
    __syncthreads();

    // ---- inclusive XOR scan of the tile, seeded with the carry ----
    uint32_t q = (nwords + T - 1) / T;
    q |= 1u;  // odd stride between threads' segments avoids LDS bank conflicts
    const uint32_t w0 = min(tid * q, nwords), w1 = min(w0 + q, nwords);
    uint32_t red = 0;
    for (uint32_t w = w0; w < w1; w++) red ^= lw[w];
    red ^= red >> 16;
    red ^= red >> 8;
    red &= 0xFFu;
    uint32_t total;
    const uint32_t excl = block_xor_scan_excl(red, scan_sh, total);
    uint32_t c = (carry_sh ^ excl) & 0xFFu;
    for (uint32_t w = w0; w < w1; w++) {
      uint32_t p = lw[w];
      p ^= p << 8;
      p ^= p << 16;
      p ^= c * 0x01010101u;
      lw[w] = p;
      c = p >> 24;
    }
    __syncthreads();
    if (tid == 0) carry_sh = lds[St - 1];

    // ---- write the cipher rows of the tile ----
    uint8_t* dt = dst + (uint64_t)t0 * row;
    for (uint32_t w = tid; w < nwords; w += T) store_bytes(dt + 4 * w, lw[w], min(4u, St - 4 * w));
    __syncthreads();
  }
}

// ------------------------------------------------------------ decrypt ----
__global__ __launch_bounds__(kMaxThreads) void round_dec_kernel(RoundArgs A) {
  extern __shared__ __align__(16) uint8_t lds[];
  const Geom g = A.g;
  const uint32_t tid = threadIdx.x, T = blockDim.x, frame = blockIdx.y;
  const uint64_t row = (uint64_t)g.W * g.C;
  const uint32_t t0 = blockIdx.x * A.tile_rows;
  const uint32_t R = min(A.tile_rows, g.H - t0);
  const uint8_t* src = A.src + (uint64_t)frame * A.frame_bytes;
  uint8_t* dst = A.dst + (uint64_t)frame * A.frame_bytes;
  const uint32_t* gm = A.gm + (uint64_t)frame * g.H;
  const uint8_t* ks = A.ks + (uint64_t)frame * A.ks_stride;

  // per-band tables after the tile: first row and recovered seed
  uint32_t* blo = reinterpret_cast<uint32_t*>(lds + (((uint64_t)A.tile_rows * row + 15) & ~15ull));
  uint8_t* seed = reinterpret_cast<uint8_t*>(blo + g.n + 1);
  for (uint32_t i = tid; i <= g.n; i += T) blo[i] = (uint32_t)band_lo(g.H, g.n, i);
  __syncthreads();
  for (uint32_t i = tid; i < g.n; i += T) {
    // s_d of band i = pre-diffusion last byte of band i' = (i+1) mod n,
    // recovered by Eq. (4) from that band's last two cipher bytes
    const uint32_t ip = i + 1 == g.n ? 0 : i + 1;
    const uint64_t Sp = (uint64_t)(blo[ip + 1] - blo[ip]) * row;
    const uint64_t m = (uint64_t)blo[ip + 1] * row - 1;
    const uint8_t bp = ks[(uint64_t)g.r * blo[ip] * row + (uint64_t)A.j * Sp + Sp - 1];
    seed[i] = (uint8_t)((bp ^ src[m] ^ src[m - 1]) - bp);
  }
  __syncthreads();

  const uint32_t M = (g.W + g.H - 1) / g.H;
  const uint32_t nslots = T / R;
  const uint32_t k = tid % R, slot = tid / R;
  if (slot < nslots) {
    const uint32_t a = t0 + k;  // destination (plain) row
    uint8_t* drow = lds + (uint64_t)k * row;
    uint32_t bi = 0;            // band of alpha, advanced monotonically
    for (uint32_t alpha = slot; alpha < g.H; alpha += nslots) {
      while (blo[bi + 1] <= alpha) bi++;
      const uint64_t band_start = (uint64_t)blo[bi] * row;
      const uint64_t Sb = (uint64_t)(blo[bi + 1] - blo[bi]) * row;
      // keystream byte of flat position x: block of band bi, round j
      const uint8_t* kb = ks + (uint64_t)g.r * band_start + (uint64_t)A.j * Sb;
      const uint32_t shift = gm[alpha];
      uint32_t ob = alpha + g.H - a;
      if (ob >= g.H) ob -= g.H;
      for (uint32_t m = 0; m < M; m++) {
        const uint32_t o = ob + m * g.H;
        if (o >= g.W) break;
        uint32_t beta = o + shift;
        if (beta >= g.W) beta -= g.W;
        const uint64_t x = ((uint64_t)alpha * g.W + beta) * g.C;
        uint8_t prev = x == band_start ? seed[bi] : src[x - 1];
        uint8_t* dp = drow + (uint64_t)o * g.C;
        for (uint32_t c = 0; c < g.C; c++) {
          const uint8_t z = src[x + c], b = kb[x + c - band_start];
          dp[c] = (uint8_t)((b ^ z ^ prev) - b);
          prev = z;
        }
      }
    }
  }
  __syncthreads();
  const uint32_t St = R * (uint32_t)row;
  const uint32_t nwords = (St + 3) / 4;
  const uint32_t* lw = reinterpret_cast<const uint32_t*>(lds);
  uint8_t* dt = dst + (uint64_t)t0 * row;
  for (uint32_t w = tid; w < nwords; w += T) store_bytes(dt + 4 * w, lw[w], min(4u, St - 4 * w));
}

}  // namespace

size_t round_lds_bytes(const Geom& g, uint32_t tile_rows) {
  const size_t tile = (((size_t)tile_rows * g.W * g.C) + 15) & ~(size_t)15;
  return tile + 4 * ((size_t)g.n + 1) + g.n + 16;
}

hipError_t launch_round_enc(const RoundArgs& a, uint32_t threads, hipStream_t s) {
  const size_t lds = round_lds_bytes(a.g, a.tile_rows);
  hipLaunchKernelGGL(round_enc_kernel, dim3(a.g.n, a.n_frames), dim3(threads), lds, s, a);
  return hipGetLastError();
}

hipError_t launch_round_dec(const RoundArgs& a, uint32_t threads, hipStream_t s) {
  const size_t lds = round_lds_bytes(a.g, a.tile_rows);
  const uint32_t tiles = (a.g.H + a.tile_rows - 1) / a.tile_rows;
  hipLaunchKernelGGL(round_dec_kernel, dim3(tiles, a.n_frames), dim3(threads), lds, s, a);
  return hipGetLastError();
}

}  // namespace cv
