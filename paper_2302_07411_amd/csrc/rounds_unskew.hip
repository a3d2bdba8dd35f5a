// All r decryption rounds of a batch of frames (Sec. 2, Eq. (4) then
// Eq. (2), rounds in reverse order), for frames whose every band fits the LDS
// as one tile.
//
// Round j of a band: its input Z_j (the cipher for j = r-1, else the output
// of round j+1) is taken in chain order and Eq. (4) undone byte by byte,
// Y_k = (b_k ^ Z_k ^ Z_{k-1}) - b_k mod 256: element-wise once the
// predecessor Z_{k-1} is known, so every lane takes 4 consecutive pixels
// (12 or 16 bytes) of the band with 12- or 16-byte loads of its keystream at
// a 12- or 16-byte lane stride (coalesced), reads the byte before its pixels
// directly, and stores its Y words to the group's scratch frame, also
// coalesced.  The seed Z_{-1} of band i is the pre-diffusion last byte of
// band i+1, recovered from that band's last two bytes of Z_j (Eq. 4 again).
//
// Then Eq. (2): X[a][o] = Y[alpha][beta] with alpha = (a+o) mod H,
// beta = (o + g(alpha)) mod W.  Seen from the band's rows, source row alpha
// contributes R consecutive pixels beta (one per band row, beta falling as
// the row rises), so the gather reads every source row as a contiguous run
// (coalesced) and writes the band's tile T[k][o] along a diagonal (LDS words
// pitch-1 apart: across banks).  The tile holds X_j = Z_{j-1} for the band in
// row order, which is exactly what the next round's Eq. (4) reads; the
// last round's tile is the plaintext band, stored packed.
//
// Workgroups form groups of n (one per band) that walk frames; one group
// barrier per round separates the scratch writes of Eq. (4) from the
// gathers of Eq. (2).  Two scratch frames alternate round after round (also
// across frames), so no round writes the frame that a slower member may
// still be gathering from.
#include "tile_ops.h"

namespace cv {
namespace {

using namespace tile;

constexpr uint32_t kThreads = 1024;
constexpr uint32_t kPitchPad = 4;   // LDS row pitch W+4: 16-byte aligned rows, odd diagonal stride
constexpr uint32_t kGatherBatch = 8;
constexpr uint32_t kPassBatch = 3;  // passes of Eq. (4) whose loads are issued together

struct UnskewArgs {
  const uint8_t* in;       // cipher frames (packed)
  uint8_t* out;            // plaintext frames (packed)
  const uint8_t* ks;       // keystream (packed, canonical), frame after frame
  const uint32_t* gm;      // shift tables g(alpha) mod W, H per frame
  uint8_t* scratch;        // per group: two pixel-word frames
  uint32_t* counters;      // per group one 128-byte line: barrier counter, XCC id
  uint32_t* err;
  Geom g;
  uint32_t n_frames, groups, spin_limit;
};

// C bytes per pixel as 12- or 16-byte global accesses that are only
// 4-byte aligned.
typedef uint32_t v3u32a4 __attribute__((ext_vector_type(3), aligned(4)));
typedef __attribute__((address_space(1))) const v3u32a4 gcv3a4;
typedef __attribute__((address_space(1))) v3u32a4 gv3a4;
typedef __attribute__((address_space(1))) v4u32a4 gv4a4;

template <uint32_t C>
__device__ __forceinline__ void load_run(const uint8_t* p, uint32_t* w) {
  if constexpr (C == 3) {
    const v3u32a4 x = *(gcv3a4*)p;
    w[0] = x.x;
    w[1] = x.y;
    w[2] = x.z;
  } else {
    const v4u32a4 x = gload4u(p);
    w[0] = x.x;
    w[1] = x.y;
    w[2] = x.z;
    w[3] = x.w;
  }
}

template <uint32_t C>
__device__ __forceinline__ void store_run(uint8_t* p, const uint32_t* w) {
  if constexpr (C == 3) {
    v3u32a4 x;
    x.x = w[0];
    x.y = w[1];
    x.z = w[2];
    *(gv3a4*)p = x;
  } else {
    v4u32a4 x;
    x.x = w[0];
    x.y = w[1];
    x.z = w[2];
    x.w = w[3];
    *(gv4a4*)p = x;
  }
}

// Seed of Eq. (4) from a band's last two bytes z1 (last) and z0 and its
// keystream byte b at the last position: the pre-diffusion last byte.
__device__ __forceinline__ uint32_t seed_of(uint32_t z1, uint32_t z0, uint32_t b) {
  return ((b ^ z1 ^ z0) - b) & 0xFFu;
}

// Eq. (4) over the band's chain: pass p, lane t takes run q = p*kThreads + t
// (pixels 4q..4q+3 of the band).  Z comes from the packed cipher band `zin`
// (first round) or from the LDS tile (pixel words, row pitch `pitch`).
// Y goes to the scratch frame `ybuf` as pixel words at the band's pixels.
template <uint32_t C, bool kFromGlobal>
__device__ __forceinline__ void undiffuse_band(const uint8_t* zin, const uint32_t* tile,
                                               uint32_t pitch, const uint8_t* kb, uint32_t W,
                                               uint32_t npix, uint32_t seed, uint32_t* ybuf) {
  constexpr uint32_t DW = C;  // words per run of 4 pixels (packed bytes)
  const uint32_t nruns = npix / 4;
  for (uint32_t q0 = threadIdx.x; q0 < nruns; q0 += kPassBatch * kThreads) {
    uint32_t Z[kPassBatch][DW], K[kPassBatch][DW], pred[kPassBatch];
#pragma unroll
    for (uint32_t u = 0; u < kPassBatch; u++) {
      const uint32_t q = q0 + u * kThreads;
      const uint32_t qc = q < nruns ? q : 0u;
      load_run<C>(kb + (uint64_t)qc * 4 * C, K[u]);
      if constexpr (kFromGlobal) {
        load_run<C>(zin + (uint64_t)qc * 4 * C, Z[u]);
        pred[u] = qc > 0 ? g32(zin + (uint64_t)qc * 4 * C - 4)[0] : 0u;
      } else {
        const uint32_t k = (4 * qc) / W, c = 4 * qc - k * W;
        const uint4 y = *reinterpret_cast<const uint4*>(tile + k * pitch + c);
        const uint32_t w4[4] = {y.x, y.y, y.z, y.w};
        if constexpr (C == 3) {
          pack4(w4, Z[u]);
        } else {
#pragma unroll
          for (uint32_t e = 0; e < 4; e++) Z[u][e] = w4[e];
        }
        // the pixel before the run: same row, or the last of the row above
        const uint32_t pk = c > 0 ? k : k - 1, pc = c > 0 ? c - 1 : W - 1;
        pred[u] = qc > 0 ? tile[pk * pitch + pc] << (8 * (4 - C)) : 0u;
      }
    }
#pragma unroll
    for (uint32_t u = 0; u < kPassBatch; u++) {
      const uint32_t q = q0 + u * kThreads;
      if (q >= nruns) break;
      // predecessor bytes: Z shifted up by one byte, the first from pred
      uint32_t prev = q > 0 ? pred[u] : seed << 24;
      uint32_t Y[DW];
#pragma unroll
      for (uint32_t i = 0; i < DW; i++) {
        const uint32_t zp = __builtin_amdgcn_alignbyte(Z[u][i], prev, 3);
        Y[i] = sub_bytes(K[u][i] ^ Z[u][i] ^ zp, K[u][i]);
        prev = Z[u][i];
      }
      uint32_t w4[4];
      if constexpr (C == 3) {
        unpack4(Y, w4);
      } else {
#pragma unroll
        for (uint32_t e = 0; e < 4; e++) w4[e] = Y[e];
      }
      gstore4(ybuf + 4 * (uint64_t)q, make_uint4(w4[0], w4[1], w4[2], w4[3]));
    }
  }
}

// Eq. (2) for the band's rows [t0, t0+R): T[k][o] = Y[alpha][beta] with
// alpha = (t0+k+o) mod H, beta = (o + g(alpha)) mod W.  Thread (k, m) walks
// source rows alpha = s, s+A, ...; its pixel of row alpha is column
// o = (alpha - t0 - k) mod H (+ m*H).  gsh: the frame's shift table in LDS.
template <bool kFull>
__device__ __forceinline__ void unskew_gather(const uint32_t* Y, const Geom& g, uint32_t t0,
                                              uint32_t R, const uint32_t* gsh, uint32_t* tile,
                                              uint32_t pitch) {
  const uint32_t W = g.W, H = g.H;
  const uint32_t M = (W + H - 1) / H;  // runs per source row
  const uint32_t per = R * M;
  const uint32_t A = kThreads / per;   // source rows walked side by side
  const uint32_t t = threadIdx.x;
  if (t >= per * A) return;
  const uint32_t k = t % R, rest = t / R, m = rest % M, s = rest / M;
  const uint32_t mH = m * H;
  uint32_t* row = tile + k * pitch;
  for (uint32_t al0 = s; al0 < H; al0 += kGatherBatch * A) {
    uint32_t val[kGatherBatch];
#pragma unroll
    for (uint32_t u = 0; u < kGatherBatch; u++) {
      const uint32_t al = al0 + u * A;
      const uint32_t alc = al < H ? al : 0u;
      const int32_t d = (int32_t)alc - (int32_t)(t0 + k);
      const uint32_t o = (d < 0 ? (uint32_t)(d + (int32_t)H) : (uint32_t)d) + mH;
      const bool ok = al < H && (kFull || o < W);
      uint32_t beta = o + gsh[alc];
      if (beta >= W) beta -= W;
      val[u] = g32(Y)[ok ? (uint64_t)alc * W + beta : 0u];
    }
#pragma unroll
    for (uint32_t u = 0; u < kGatherBatch; u++) {
      const uint32_t al = al0 + u * A;
      const uint32_t alc = al < H ? al : 0u;
      const int32_t d = (int32_t)alc - (int32_t)(t0 + k);
      const uint32_t o = (d < 0 ? (uint32_t)(d + (int32_t)H) : (uint32_t)d) + mH;
      if (al < H && (kFull || o < W)) row[o] = val[u];
    }
  }
}

template <uint32_t C, bool kFull>
__global__ __launch_bounds__(kThreads) void rounds_unskew_kernel(UnskewArgs A) {
  extern __shared__ __align__(16) uint32_t lds[];
  __shared__ uint32_t seed_sh;
  const Geom g = A.g;
  const uint32_t W = g.W, H = g.H, n = g.n, r = g.r;
  // XCD-aware placement: workgroup i runs on XCD i % 8; group members share it
  const uint32_t i = blockIdx.x, xcd = i % 8, idx = i / 8;
  const uint32_t group = xcd + 8 * (idx / n), band = idx % n;
  if (group >= A.groups) return;
  const uint64_t pwf = (uint64_t)H * W * 4, F = (uint64_t)H * W * C;
  uint32_t* buf[2] = {(uint32_t*)(A.scratch + (uint64_t)group * 2 * pwf),
                      (uint32_t*)(A.scratch + (uint64_t)group * 2 * pwf + pwf)};
  uint32_t* ctr = A.counters + 32 * group;
  check_group_xcc(ctr + 1, A.err);
  const uint32_t lo = (uint32_t)band_lo(H, n, band), hi = (uint32_t)band_lo(H, n, band + 1);
  const uint32_t R = hi - lo, npix = R * W;
  const uint64_t S = (uint64_t)npix * C;
  const uint32_t pitch = W + kPitchPad;
  uint32_t* tile = lds;
  uint32_t* gsh = lds + R * pitch;
  // the next band, whose last two bytes seed this band
  const uint32_t nb = band + 1 == n ? 0 : band + 1;
  const uint32_t nlo = (uint32_t)band_lo(H, n, nb), nhi = (uint32_t)band_lo(H, n, nb + 1);
  const uint64_t nS = (uint64_t)(nhi - nlo) * W * C;
  uint32_t nbar = 0, turn = 0;
  for (uint32_t f = group; f < A.n_frames; f += A.groups) {
    const uint8_t* ks = A.ks + (uint64_t)f * r * F;
    const uint8_t* kband = ks + (uint64_t)r * lo * W * C;           // this band's r*S bytes
    const uint8_t* knext = ks + (uint64_t)r * nlo * W * C;          // band nb's
    const uint8_t* cin = A.in + (uint64_t)f * F;
    __syncthreads();  // every thread is done with the previous frame's table and tile
    for (uint32_t a = threadIdx.x; a < H; a += kThreads) gsh[a] = A.gm[(uint64_t)f * H + a];
    if (threadIdx.x == 0) {
      // seed of round r-1: band nb's last two cipher bytes
      const uint64_t e = (uint64_t)nhi * W * C;
      const uint32_t z1 = ((const gcu8*)cin)[e - 1], z0 = ((const gcu8*)cin)[e - 2];
      seed_sh = seed_of(z1, z0, ((const gcu8*)knext)[(uint64_t)(r - 1) * nS + nS - 1]);
    }
    __syncthreads();
    for (uint32_t jj = 0; jj < r; jj++) {
      const uint32_t j = r - 1 - jj;
      uint32_t* ybuf = buf[turn];
      turn ^= 1;
      const uint32_t seed = seed_sh;
      // Eq. (4) on the band: Z_j in chain order -> Y_j into the scratch frame
      if (jj == 0)
        undiffuse_band<C, true>(cin + (uint64_t)lo * W * C, tile, pitch, kband + (uint64_t)j * S, W,
                                npix, seed, ybuf + (uint64_t)lo * W);
      else
        undiffuse_band<C, false>(nullptr, tile, pitch, kband + (uint64_t)j * S, W, npix, seed,
                                 ybuf + (uint64_t)lo * W);
      nbar++;
      if (!group_barrier(ctr, nbar * n, A.spin_limit, A.err)) return;
      // Eq. (2): the band's rows of X_j from every band's Y_j
      unskew_gather<kFull>(ybuf, g, lo, R, gsh, tile, pitch);
      if (j > 0 && threadIdx.x == 0) {
        // seed of round j-1: band nb's last pixel of X_j, i.e. Y_j at its
        // position under Eq. (2)
        const uint32_t a = nhi - 1, o = W - 1;
        const uint32_t al = (a + o) % H;
        uint32_t beta = o + gsh[al];
        if (beta >= W) beta -= W;
        const uint32_t y = g32(ybuf)[(uint64_t)al * W + beta];
        const uint32_t z1 = (y >> (8 * (C - 1))) & 0xFFu, z0 = (y >> (8 * (C - 2))) & 0xFFu;
        seed_sh = seed_of(z1, z0, ((const gcu8*)knext)[(uint64_t)(j - 1) * nS + nS - 1]);
      }
      __syncthreads();
    }
    // the last round's tile is the plaintext band: store it packed
    uint8_t* dst = A.out + (uint64_t)f * F + (uint64_t)lo * W * C;
    for (uint32_t q = threadIdx.x; q < npix / 4; q += kThreads) {
      const uint32_t k = (4 * q) / W, c = 4 * q - k * W;
      const uint4 y = *reinterpret_cast<const uint4*>(tile + k * pitch + c);
      const uint32_t w4[4] = {y.x, y.y, y.z, y.w};
      uint32_t P[C];
      if constexpr (C == 3) {
        pack4(w4, P);
      } else {
#pragma unroll
        for (uint32_t e = 0; e < 4; e++) P[e] = w4[e];
      }
      store_run<C>(dst + (uint64_t)q * 4 * C, P);
    }
  }
}

__global__ void reset_unskew_groups(uint32_t* p, uint32_t groups) {
  for (uint32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < groups; k += gridDim.x * blockDim.x) {
    p[32 * k] = 0;
    p[32 * k + 1] = 0xFFFFFFFFu;
  }
}

template <uint32_t C, bool kFull>
const void* unskew_fn() {
  return reinterpret_cast<const void*>(&rounds_unskew_kernel<C, kFull>);
}

const void* pick(const Geom& g) {
  const bool full = g.W % g.H == 0;
  if (g.C == 3) return full ? unskew_fn<3, true>() : unskew_fn<3, false>();
  return full ? unskew_fn<4, true>() : unskew_fn<4, false>();
}

uint32_t max_band_rows(const Geom& g) {
  uint32_t m = 0;
  for (uint32_t i = 0; i < g.n; i++)
    m = std::max<uint32_t>(m, (uint32_t)(band_lo(g.H, g.n, i + 1) - band_lo(g.H, g.n, i)));
  return m;
}

}  // namespace

size_t rounds_unskew_lds_bytes(const Geom& g) {
  return ((size_t)max_band_rows(g) * (g.W + kPitchPad) + g.H) * 4;
}

bool rounds_unskew_applies(const Geom& g, size_t lds_max) {
  if (!((g.C == 3 || g.C == 4) && g.W % 16 == 0)) return false;
  const uint32_t M = (g.W + g.H - 1) / g.H;
  const size_t reserve = 1024;  // static LDS of the kernel and group-barrier words
  return (size_t)max_band_rows(g) * M <= kThreads &&
         rounds_unskew_lds_bytes(g) + reserve <= lds_max;
}

uint32_t rounds_unskew_resident_groups(const Geom& g, int device) {
  int per_cu = 0, cus = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, pick(g), kThreads,
                                                   rounds_unskew_lds_bytes(g)) != hipSuccess ||
      per_cu <= 0)
    return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess) return 0;
  const uint32_t per_xcd = (uint32_t)per_cu * (uint32_t)cus / 8;
  return (per_xcd / g.n) * 8;
}

hipError_t launch_rounds_unskew(const RoundsFusedArgs& r, hipStream_t s) {
  UnskewArgs a;
  a.in = r.in;
  a.out = r.out;
  a.ks = r.ks;
  a.gm = r.gm;
  a.scratch = r.scratch;
  a.counters = r.counters;
  a.err = r.err;
  a.g = r.g;
  a.n_frames = r.n_frames;
  a.groups = r.groups;
  a.spin_limit = r.spin_limit;
  hipLaunchKernelGGL(reset_unskew_groups, dim3(1), dim3(256), 0, s, r.counters, r.groups);
  const size_t lds = rounds_unskew_lds_bytes(r.g);
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
