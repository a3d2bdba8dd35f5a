// PLCM keystream generator for gfx950 (Sec. 3, Eq. (5) and the PLCM byte
// generator of the speed evaluation).
//
// Each band of each stream owns one chain: two PLCMs iterated in lockstep.
// A step yields one iterate of each map; bytes 0..5 of each iterate's
// binary64 bit pattern (least significant first, i.e. mantissa bits 0..47)
// are XORed pairwise into 6 keystream bytes.  A frame needs r*S_i bytes,
// i.e. ceil(r*S_i/6) steps; the unused bytes of the last step are dropped.
// The chain state persists across frames and calls.
//
// The chain is a strict serial recurrence, so the kernel is bound by the
// latency of one step.  A workgroup is two wavefronts on different SIMDs:
//  - the producer runs up to 32 chains, both maps of chain c in lanes 2c and
//    2c+1 (a step costs the latency of one map), and only writes each
//    iterate to an LDS ring -- one ds_write per step;
//  - the consumer turns a finished block of 32 steps into keystream bytes
//    (pair XOR, packing, 16-byte stores) while the producer runs the next
//    block.  One barrier per block hands the double-buffered ring over.
//
// Every floating-point result equals the single correctly rounded IEEE-754
// binary64 operation the map prescribes (round to nearest even; built with
// -ffp-contract=off, no fast-math).  A chaotic orbit amplifies any rounding
// difference, so this is what makes the keystream bit-identical to any other
// correct implementation.  The division x/d by a key constant d is done in
// one of two ways, with identical results:
//  - exact path: the compiler's IEEE division;
//  - fast path: y = RN(1/d) precomputed on the host, q0 = RN(x*y), then two
//    FMA corrections q <- RN(q + RN(x - d*q)*y).  After the first correction
//    q is faithful (within one ulp of x/d); Markstein's theorem (for y =
//    RN(1/d), a faithful q and the exact remainder x - d*q, RN(q + r*y) =
//    RN(x/d)) then makes the second one correctly rounded.  Its conditions
//    (normal operands, exact remainder, no underflow) hold when d >= 2^-64
//    and x is 0 or >= 2^-900; the host enables the fast path only for keys
//    with p >= 2^-64 and every state 0 or >= 2^-800, and along any orbit
//    from such a state every nonzero numerator stays >= 2^-800 (each step at
//    least doubles the folded value, and y - p is a multiple of ulp(p)).
#include "cv_internal.h"

namespace cv {
namespace {

constexpr int kBlock = 32;  // steps per ring block

// Eq. (5), one step, exact IEEE division.  x in (1/2,1] is folded to 1-x
// (exact by Sterbenz' lemma); min(x, 1-x) picks the same value.
__device__ __forceinline__ double plcm_exact(double x, double p, double h) {
  const double y = (x > 0.5) ? 1.0 - x : x;
  const bool first = y < p;
  const double num = first ? y : y - p;
  const double den = first ? p : h;
  return num / den;
}

// v_min_f64 without the NaN-canonicalising extra instruction the generic
// fmin lowers to (no NaN can occur here).
__device__ __forceinline__ double vmin(double a, double b) {
  double r;
  asm volatile("v_min_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
  return r;
}

// Eq. (5), one step, division by the selected key constant through its
// precomputed reciprocal and two FMA corrections (see the file comment).
__device__ __forceinline__ double plcm_fast(double x, double p, double h, double ip, double ih) {
  const double y = vmin(x, 1.0 - x);
  const bool first = y < p;
  const double num = first ? y : y - p;
  const double den = first ? p : h;
  const double rcp = first ? ip : ih;
  double q = num * rcp;
  double e = __builtin_fma(-den, q, num);
  q = __builtin_fma(e, rcp, q);
  e = __builtin_fma(-den, q, num);
  return __builtin_fma(e, rcp, q);
}

template <bool kFast>
__device__ __forceinline__ double plcm(double x, double p, double h, double ip, double ih) {
  if constexpr (kFast) return plcm_fast(x, p, h, ip, ih);
  return plcm_exact(x, p, h);
}

__device__ __forceinline__ uint32_t wave_max(uint32_t v) {
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) v = max(v, (uint32_t)__shfl_xor((int)v, d, 64));
  return v;
}

struct ChainPlan {
  uint64_t nbytes;   // bytes per frame
  uint32_t spf;      // steps per frame = ceil(nbytes / 6)
  uint32_t total;    // steps over all frames of this launch
};

__device__ __forceinline__ ChainPlan plan(const PlcmChain& ch, uint32_t n_frames) {
  ChainPlan c;
  c.nbytes = ch.nbytes;
  c.spf = (uint32_t)((ch.nbytes + 5) / 6);
  c.total = c.spf * n_frames;
  return c;
}

// Consumer: bytes of ring block `blk` for one chain.
__device__ void emit_block(const double* ring, uint32_t lane, uint32_t blk, const ChainPlan& cp,
                           uint8_t* base, uint64_t stride, uint32_t& f, uint32_t& sf,
                           double* state) {
  const uint32_t g0 = blk * kBlock;
  if (g0 >= cp.total) return;
  const double2* r2 = reinterpret_cast<const double2*>(ring);  // [step][chain] pairs
  // state after the last step of the launch
  const uint32_t last = cp.total - 1;
  if (last >= g0 && last < g0 + kBlock) {
    const double2 v = r2[(last - g0) * 32 + lane];
    state[0] = v.x;
    state[1] = v.y;
  }
  uint8_t* out = base + (uint64_t)f * stride;
  if ((sf & 7u) == 0 && (uint64_t)(sf + kBlock) * 6 <= cp.nbytes &&
      ((((uintptr_t)out) + (uint64_t)sf * 6) & 15u) == 0) {
    uint4* o4 = reinterpret_cast<uint4*>(out + (uint64_t)sf * 6);
#pragma unroll
    for (int t = 0; t < kBlock / 8; t++) {
      uint32_t w[12];
#pragma unroll
      for (int s = 0; s < 4; s++) {
        const double2 a = r2[(t * 8 + 2 * s) * 32 + lane];
        const double2 b = r2[(t * 8 + 2 * s + 1) * 32 + lane];
        const uint64_t u = (uint64_t)__double_as_longlong(a.x) ^ (uint64_t)__double_as_longlong(a.y);
        const uint64_t v = (uint64_t)__double_as_longlong(b.x) ^ (uint64_t)__double_as_longlong(b.y);
        w[3 * s + 0] = (uint32_t)u;
        w[3 * s + 1] = ((uint32_t)(u >> 32) & 0xFFFFu) | ((uint32_t)v << 16);
        w[3 * s + 2] = ((uint32_t)v >> 16) | ((uint32_t)(v >> 32) << 16);
      }
      o4[3 * t + 0] = make_uint4(w[0], w[1], w[2], w[3]);
      o4[3 * t + 1] = make_uint4(w[4], w[5], w[6], w[7]);
      o4[3 * t + 2] = make_uint4(w[8], w[9], w[10], w[11]);
    }
    sf += kBlock;
    if (sf == cp.spf) {
      sf = 0;
      f++;
    }
    return;
  }
  // general path: step by step, frame boundaries and partial last steps
  for (uint32_t s = 0; s < (uint32_t)kBlock && g0 + s < cp.total; s++) {
    const double2 a = r2[s * 32 + lane];
    const uint64_t u = (uint64_t)__double_as_longlong(a.x) ^ (uint64_t)__double_as_longlong(a.y);
    const uint64_t at = (uint64_t)sf * 6;
    const uint64_t left = cp.nbytes - at;
    const int take = left < 6 ? (int)left : 6;
    uint8_t* o = base + (uint64_t)f * stride + at;
    for (int k = 0; k < take; k++) o[k] = (uint8_t)(u >> (8 * k));
    if (++sf == cp.spf) {
      sf = 0;
      f++;
    }
  }
}

template <bool kFast>
__global__ __launch_bounds__(128) void prbg_plcm_kernel(const PlcmChain* __restrict__ chains,
                                                         uint32_t n_chains, uint8_t* ks_base,
                                                         uint32_t n_frames) {
  __shared__ double ring[2][kBlock * 64];  // [buf][step][lane]
  const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
  const uint32_t c0 = blockIdx.x * 32u;
  const uint32_t nch = min(32u, n_chains - c0);

  // chain of this lane: producer lane 2c+m -> chain c, map m; consumer lane c
  const uint32_t my_c = wave == 0 ? (lane >> 1) : lane;
  const bool has = my_c < nch;
  PlcmChain ch{};
  if (has) ch = chains[c0 + my_c];
  const ChainPlan cp = plan(ch, n_frames);
  const uint32_t total_max = wave_max(has ? cp.total : 0u);
  const uint32_t nblk = (total_max + kBlock - 1) / kBlock;

  if (wave == 0) {
    const uint32_t m = lane & 1u;
    const double p = ch.p[m], h = ch.h[m], ip = ch.ip[m], ih = ch.ih[m];
    double x = has ? ch.state[m] : 0.0;
    for (uint32_t b = 0; b < nblk; b++) {
      double* dst = &ring[b & 1u][lane];
#pragma unroll
      for (int s = 0; s < kBlock; s++) {
        x = plcm<kFast>(x, p, h, ip, ih);
        dst[s * 64] = x;
      }
      __syncthreads();
    }
  } else {
    uint32_t f = 0, sf = 0;
    uint8_t* base = ks_base + ch.out_off;
    for (uint32_t b = 0; b < nblk; b++) {
      if (b > 0 && has) emit_block(ring[(b - 1) & 1u], lane, b - 1, cp, base, ch.frame_stride, f,
                                   sf, ch.state);
      __syncthreads();
    }
    if (nblk > 0 && has)
      emit_block(ring[(nblk - 1) & 1u], lane, nblk - 1, cp, base, ch.frame_stride, f, sf,
                 ch.state);
  }
}

}  // namespace

hipError_t launch_prbg_plcm(const PlcmChain* d_chains, uint32_t n_chains, uint8_t* ks_base,
                            uint32_t n_frames, bool fast, hipStream_t s) {
  if (n_chains == 0 || n_frames == 0) return hipSuccess;
  const uint32_t blocks = (n_chains + 31) / 32;
  if (fast)
    hipLaunchKernelGGL(prbg_plcm_kernel<true>, dim3(blocks), dim3(128), 0, s, d_chains, n_chains,
                       ks_base, n_frames);
  else
    hipLaunchKernelGGL(prbg_plcm_kernel<false>, dim3(blocks), dim3(128), 0, s, d_chains, n_chains,
                       ks_base, n_frames);
  return hipGetLastError();
}

}  // namespace cv
