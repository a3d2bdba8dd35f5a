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
//    2c+1 (a step costs the latency of one map), and only writes its
//    iterates to an LDS ring, two steps per 16-byte write (every memory
//    instruction costs the chain issue time, so they are kept few and wide);
//  - the consumer turns a finished block of 32 steps into keystream bytes
//    (pair XOR, packing, 16-byte stores), the block split over all its
//    lanes, while the producer runs the next block.  One barrier per block
//    hands the double-buffered ring over.
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
// With the fast path, each map can also be given two lanes, one per piece of
// Eq. (5): lane A always divides y by p, lane B always divides y-p by 1/2-p,
// so neither selects its operands; a DPP swap then lets both lanes take the
// candidate of the piece y actually falls in.  This shortens the dependent
// chain of a step; 16 chains fit a wavefront.
//
// The speculative variant shortens the chain further.  With zh = RN(1/d) and
// zl = RN(1/d - zh) precomputed, q = RN(zh*y + RN(zl*y)) is one multiply and
// one FMA; zh + zl carries 1/d to about 2^-106 relative, so q is within one
// ulp of y/d and equals RN(y/d) unless y/d lies within about 2^-105 (relative)
// of a rounding midpoint.  Such quotients exist but are extremely rare (none
// in 2e8 orbit steps, none in 2e6 quotients constructed next to midpoints),
// and correctness may not rest on rarity: the producer wavefront runs the
// map with this quotient and keeps only a few checkpoints per block; three
// verifier wavefronts recompute the block's steps from the checkpoints with
// the same operations, check every step against its predecessor (the
// remainder by one FMA and one Markstein correction must give the value
// back, see plcm_wrong_yg) and the producer's checkpoints against their own
// values; an emitter wavefront turns verified blocks into bytes.  On a
// mismatch every wavefront takes a repair branch: the producer recomputes
// the failed block and the one after it with the correctly rounded fast path
// above.  The checks run on other SIMDs while the producer iterates, and the
// producer writes to LDS only three times per block, so the chain runs at
// the producer's own issue rate: seven FP64 instructions per step.
#include "cv_internal.h"

namespace cv {
namespace {

constexpr int kBlock = 32;  // steps per ring block
constexpr uint32_t kSpecVerifiers = 3;  // verifier wavefronts of the speculative generator
                                        // (two are too slow for the producer; more than
                                        // three put a fourth wavefront on a shared SIMD)

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

// Value of the same 64-bit register in the adjacent lane (0<->1, 2<->3, ...),
// DPP quad_perm(1,0,3,2); the partner lane is always active.
__device__ __forceinline__ double swap_pair(double v) {
  const uint64_t u = (uint64_t)__double_as_longlong(v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)u, 0xB1, 0xF, 0xF, true);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)(u >> 32), 0xB1, 0xF, 0xF, true);
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// One lane of a per-piece pair: `off`, `den`, `rcp` are this lane's piece
// (lane A: 0, p, 1/p; lane B: p, 1/2-p, 1/(1/2-p)); `lane_b` says which.
// Both lanes of the pair return the same next iterate.
__device__ __forceinline__ double plcm_pair(double x, double p, double off, double den,
                                            double rcp, bool lane_b) {
  const double y = vmin(x, 1.0 - x);
  const double num = y - off;  // exact 0 offset on lane A
  double q = num * rcp;
  double e = __builtin_fma(-den, q, num);
  q = __builtin_fma(e, rcp, q);
  e = __builtin_fma(-den, q, num);
  q = __builtin_fma(e, rcp, q);
  const double other = swap_pair(q);
  const bool first = y < p;  // y in [0,p): first piece
  return (first != lane_b) ? q : other;
}

// Eq. (5), one step, division by the two-operation quotient of the file
// comment: both pieces are evaluated and the one y falls in is selected, so
// the dependent chain is 1-x, min, y-p, multiply, FMA, select.
__device__ __forceinline__ double plcm_two(double x, double p, double zp, double lp, double zh,
                                           double lh) {
  const double y = vmin(x, 1.0 - x);
  const double g = y - p;
  const double q1 = __builtin_fma(zp, y, lp * y);
  const double q2 = __builtin_fma(zh, g, lh * g);
  // select q1 when y < p, i.e. when g is negative (g = +0 when y = p): a
  // mask from g's sign bit and two bit-field inserts, so the select does not
  // wait for a compare (measured 1% faster on the chain than the compare)
  uint32_t m, lo, hi;
  asm("v_ashrrev_i32 %0, 31, %1" : "=v"(m) : "v"(__double2hiint(g)));
  asm("v_bfi_b32 %0, %1, %2, %3" : "=v"(lo) : "v"(m), "v"(__double2loint(q1)), "v"(__double2loint(q2)));
  asm("v_bfi_b32 %0, %1, %2, %3" : "=v"(hi) : "v"(m), "v"(__double2hiint(q1)), "v"(__double2hiint(q2)));
  return __hiloint2double((int)hi, (int)lo);
}

// Division variants of the generator (identical bytes).
enum : int { kExact = 0, kRecip = 1, kRecipPair = 2 };

template <int kMode>
__device__ __forceinline__ double plcm(double x, double p, double h, double ip, double ih) {
  if constexpr (kMode == kRecip) return plcm_fast(x, p, h, ip, ih);
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
  if (n_frames == 0) n_frames = ch.frames;
  c.nbytes = ch.nbytes;
  c.spf = (uint32_t)((ch.nbytes + 5) / 6);
  c.total = c.spf * n_frames;
  return c;
}

// Ring layout: per buffer kBlock/2 rows of 64 lanes, each slot 16 bytes
// holding one producer lane's iterates of two consecutive steps.  Chain c's
// map 1 lives in producer lane kLanes*c, map 2 in lane kLanes*c + kLanes/2.
template <uint32_t kLanes>
__device__ __forceinline__ uint64_t ring_xor(const double2* ring, uint32_t s, uint32_t c) {
  const double2 a = ring[(s >> 1) * 64 + kLanes * c];
  const double2 b = ring[(s >> 1) * 64 + kLanes * c + kLanes / 2];
  const double x1 = (s & 1) ? a.y : a.x, x2 = (s & 1) ? b.y : b.x;
  return (uint64_t)__double_as_longlong(x1) ^ (uint64_t)__double_as_longlong(x2);
}

// Per consumer lane: which frame and step-in-frame its next sub-block starts at.
struct Cursor {
  uint32_t f, sf;
};

__device__ __forceinline__ void advance(Cursor& cu, uint32_t steps, uint32_t spf) {
  cu.sf += steps;
  while (cu.sf >= spf) {
    cu.sf -= spf;
    cu.f++;
  }
}

// Consumer lane q (of kLanes per chain) of chain c: steps [q*kSub, (q+1)*kSub)
// of ring block `blk` become keystream bytes.
template <uint32_t kLanes, uint32_t kB = kBlock>
__device__ void emit_sub(const double2* ring, uint32_t c, uint32_t q, uint32_t blk,
                         const ChainPlan& cp, uint8_t* base, uint64_t stride, Cursor& cu,
                         double* state) {
  constexpr uint32_t kSub = kB / kLanes;  // steps per consumer lane
  const uint32_t s0 = q * kSub;
  const uint32_t g0 = blk * kB + s0;     // global step of the sub-block start
  if (g0 < cp.total) {
    const uint32_t last = cp.total - 1;      // state after the launch's last step
    if (last >= g0 && last < g0 + kSub) {
      const uint32_t s = s0 + (last - g0);
      const double2 a = ring[(s >> 1) * 64 + kLanes * c];
      const double2 b = ring[(s >> 1) * 64 + kLanes * c + kLanes / 2];
      state[0] = (s & 1) ? a.y : a.x;
      state[1] = (s & 1) ? b.y : b.x;
    }
    uint8_t* out = base + (uint64_t)cu.f * stride + (uint64_t)cu.sf * 6;
    if ((cu.sf & 7u) == 0 && (uint64_t)(cu.sf + kSub) * 6 <= cp.nbytes &&
        (((uintptr_t)out) & 15u) == 0) {
      uint4* o4 = reinterpret_cast<uint4*>(out);
#pragma unroll
      for (uint32_t t = 0; t < kSub / 8; t++) {
        uint32_t w[12];
#pragma unroll
        for (uint32_t u = 0; u < 4; u++) {
          const uint64_t x = ring_xor<kLanes>(ring, s0 + 8 * t + 2 * u, c);
          const uint64_t y = ring_xor<kLanes>(ring, s0 + 8 * t + 2 * u + 1, c);
          w[3 * u + 0] = (uint32_t)x;
          w[3 * u + 1] = ((uint32_t)(x >> 32) & 0xFFFFu) | ((uint32_t)y << 16);
          w[3 * u + 2] = ((uint32_t)y >> 16) | ((uint32_t)(y >> 32) << 16);
        }
        o4[3 * t + 0] = make_uint4(w[0], w[1], w[2], w[3]);
        o4[3 * t + 1] = make_uint4(w[4], w[5], w[6], w[7]);
        o4[3 * t + 2] = make_uint4(w[8], w[9], w[10], w[11]);
      }
    } else {
      // general path: step by step across frame ends and partial last steps
      Cursor v = cu;
      for (uint32_t s = 0; s < kSub && g0 + s < cp.total; s++) {
        const uint64_t x = ring_xor<kLanes>(ring, s0 + s, c);
        const uint64_t at = (uint64_t)v.sf * 6;
        const uint64_t left = cp.nbytes - at;
        const int take = left < 6 ? (int)left : 6;
        uint8_t* o = base + (uint64_t)v.f * stride + at;
        for (int k = 0; k < take; k++) o[k] = (uint8_t)(x >> (8 * k));
        advance(v, 1, cp.spf);
      }
    }
  }
  advance(cu, kB, cp.spf);
}

template <int kMode>
__global__ __launch_bounds__(128) void prbg_plcm_kernel(const PlcmChain* __restrict__ chains,
                                                         uint32_t n_chains, uint8_t* ks_base,
                                                         uint32_t n_frames) {
  // lanes per chain, in the producer and in the consumer: 2 (one per map) or
  // 4 (per map, one per piece of Eq. 5)
  constexpr uint32_t kLanes = kMode == kRecipPair ? 4 : 2;
  constexpr uint32_t kChains = 64 / kLanes;
  __shared__ double2 ring[2][(kBlock / 2) * 64];
  const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
  const uint32_t c0 = blockIdx.x * kChains;
  const uint32_t nch = min(kChains, n_chains - c0);
  const uint32_t c = lane / kLanes;
  const bool has = c < nch;
  PlcmChain ch{};
  if (has) ch = chains[c0 + c];
  const ChainPlan cp = plan(ch, n_frames);
  const uint32_t total_max = wave_max(has ? cp.total : 0u);  // same in both wavefronts
  const uint32_t nblk = (total_max + kBlock - 1) / kBlock;
  // Both wavefronts run a latency-bound chain: ask the SIMD arbiter to issue
  // them ahead of throughput work (a rounds kernel) sharing the compute unit.
  __builtin_amdgcn_s_setprio(3);

  if (wave == 0) {
    const uint32_t m = (lane / (kLanes / 2)) & 1u;
    const double p = m ? ch.p[1] : ch.p[0], h = m ? ch.h[1] : ch.h[0];
    const double ip = m ? ch.ip[1] : ch.ip[0], ih = m ? ch.ih[1] : ch.ih[0];
    double x = has ? ch.state[m] : 0.0;
    const bool lane_b = lane & 1u;
    const double off = lane_b ? p : 0.0, den = lane_b ? h : p, rcp = lane_b ? ih : ip;
    for (uint32_t b = 0; b < nblk; b++) {
      double2* dst = &ring[b & 1u][lane];
#pragma unroll
      for (int s = 0; s < kBlock; s += 2) {
        double x0;
        if constexpr (kMode == kRecipPair) {
          x0 = plcm_pair(x, p, off, den, rcp, lane_b);
          x = plcm_pair(x0, p, off, den, rcp, lane_b);
        } else {
          x0 = plcm<kMode>(x, p, h, ip, ih);
          x = plcm<kMode>(x0, p, h, ip, ih);
        }
        dst[(s / 2) * 64] = make_double2(x0, x);
      }
      __syncthreads();
    }
  } else {
    const uint32_t q = lane % kLanes;
    Cursor cu{0, 0};
    advance(cu, q * (kBlock / kLanes), cp.spf ? cp.spf : 1);
    uint8_t* base = ks_base + ch.out_off;
    for (uint32_t b = 0; b < nblk; b++) {
      if (b > 0 && has)
        emit_sub<kLanes>(ring[(b - 1) & 1u], c, q, b - 1, cp, base, ch.frame_stride, cu,
                         ch.state);
      __syncthreads();
    }
    if (nblk > 0 && has)
      emit_sub<kLanes>(ring[(nblk - 1) & 1u], c, q, nblk - 1, cp, base, ch.frame_stride, cu,
                       ch.state);
  }
}

// Speculative generator (see the file comment).  Workgroup of 2 + kNV
// wavefronts with the roles producer, emitter and kNV verifiers, assigned at
// launch from the SIMD each wavefront landed on (the producer alone on its
// SIMD).  Lane 2c+m is map m of chain c in every wavefront.  The producer
// keeps only kNV checkpoints per block (the value after the last step of each
// verifier's segment); verifier v recomputes its segment from the preceding
// checkpoint with the same two-operation step (bit-identical), writes the
// values to the ring, checks every step (plcm_wrong_yg, reusing the fold)
// and that its last value equals the producer's checkpoint, which catches a
// producer that diverged anywhere in the segment.  Iteration b: the producer
// runs block b, the verifiers block b-1, the emitter block b-2; a barrier;
// then, if a verifier reported a failure, the repair: the producer recomputes
// blocks b-1 and b from the verified end of block b-2 with the correctly
// rounded path, and every wavefront notes that block b was repaired, so that
// its verifiers skip it.  Blocks are emitted only after they are verified or
// repaired.

// Testing only: whether step `pos` of lane `lane` receives a planted error.
__device__ __forceinline__ bool planted(uint32_t pos, uint32_t lane, uint32_t period) {
  return (pos + 7 * lane) % period == 0;
}

__device__ __forceinline__ uint32_t ring_index(uint32_t s, uint32_t lane) {
  return ((s >> 1) * 64 + lane) * 2 + (s & 1u);  // as doubles: step s of a lane
}

// The two-operation step of plcm_two, also returning the fold y and y - p
// for the check below.
__device__ __forceinline__ double plcm_two_yg(double x, double p, double zp, double lp, double zh,
                                              double lh, double& y, double& g) {
  y = vmin(x, 1.0 - x);
  g = y - p;
  const double q1 = __builtin_fma(zp, y, lp * y);
  const double q2 = __builtin_fma(zh, g, lh * g);
  return y < p ? q1 : q2;
}

// Whether `cur` differs from the correctly rounded Eq. (5) step whose input
// folds to y (g = y - p), in the fast-path domain.  For each piece, the
// remainder num - cur*den by one FMA and one Markstein correction
// cur + rem*RN(1/den): if cur is within one ulp of num/den the remainder is
// exact and the correction is RN(num/den), so it equals cur exactly when cur
// is right; if cur is further away, the correction moves it by more than
// half an ulp.  Either way a wrong cur is never accepted.  (The selected
// piece's comparison decides.)
__device__ __forceinline__ bool plcm_wrong_yg(double y, double g, double cur, double p, double h,
                                              double ip, double ih) {
  double c1 = __builtin_fma(__builtin_fma(-cur, p, y), ip, cur);
  double c2 = __builtin_fma(__builtin_fma(-cur, h, g), ih, cur);
  asm("" : "+v"(c1), "+v"(c2));  // both candidates: the select stays branch-free
  return (y < p ? c1 : c2) != cur;
}

// Verifier segments: kNV-1 segments of kSegLong steps, then the rest of the
// block.  With three verifiers the last, shorter one goes to the wavefront
// that shares its SIMD with the emitter.
template <uint32_t kNV, uint32_t kB>
struct SpecSegments {
  static_assert(kB == 32 || kB == 64, "block of 32 or 64 steps");
  static constexpr uint32_t kSegLong = kNV == 3 ? (kB == 32 ? 12 : 22) : kB / kNV;
  static constexpr uint32_t kSegLast = kB - (kNV - 1) * kSegLong;
  static_assert(kSegLong % 2 == 0 && kSegLast % 2 == 0 && kSegLast <= kSegLong && kSegLast > 0,
                "segments of whole step pairs");
  // index of the checkpoint holding the value after step s, or kNV if none
  static __device__ __forceinline__ uint32_t ckpt_after(uint32_t s) {
    if (s == kB - 1) return kNV - 1;
    return (s % kSegLong == kSegLong - 1) ? s / kSegLong : kNV;
  }
};

// One verifier's segment of kLen steps from `start`: the values go to the
// ring; returns whether a step failed its check or the last value differs
// from the producer's checkpoint `end`.
template <uint32_t kLen, bool kPlant>
__device__ __forceinline__ bool verify_segment(double start, double end, double* rv, uint32_t s0,
                                               uint32_t pos0, uint32_t lane, double p, double h,
                                               double ip, double ih, double lp, double lh) {
  double val[kLen + 1], y[kLen], g[kLen];
  val[0] = start;
#pragma unroll
  for (uint32_t k = 0; k < kLen; k++) {
    double cur = plcm_two_yg(val[k], p, ip, lp, ih, lh, y[k], g[k]);
    if constexpr (kPlant)  // half of the producer's planted errors, for the per-step check
      if (planted(pos0 + k, lane, 58)) cur = __longlong_as_double(__double_as_longlong(cur) ^ 1);
    rv[ring_index(s0 + k, lane)] = cur;
    val[k + 1] = cur;
  }
  bool bad = end != val[kLen];
#pragma unroll
  for (uint32_t k = 0; k < kLen; k++) bad |= plcm_wrong_yg(y[k], g[k], val[k + 1], p, h, ip, ih);
  return bad;
}

template <bool kPlant, uint32_t kNV, uint32_t kB>
__global__ __launch_bounds__((2 + kNV) * 64) void prbg_plcm_spec_kernel(
    const PlcmChain* __restrict__ chains, uint32_t n_chains, uint8_t* ks_base, uint32_t n_frames) {
  using Seg = SpecSegments<kNV, kB>;
  constexpr uint32_t kWaves = 2 + kNV;
  __shared__ double2 ring[3][(kB / 2) * 64];  // values of blocks b-2 (emit), b-1, b (repaired)
  __shared__ double ckpt[3][kNV][64];    // per block: the value after each segment
  __shared__ uint32_t fix_count[2];      // repairs so far, of even and of odd iterations
  __shared__ uint32_t simd_of[kWaves];   // the SIMD each wavefront runs on
  const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
  const uint32_t c0 = blockIdx.x * 32;
  const uint32_t nch = min(32u, n_chains - c0);
  const uint32_t c = lane >> 1, m = lane & 1u;
  const bool has = c < nch;
  PlcmChain ch{};
  if (has) ch = chains[c0 + c];
  const ChainPlan cp = plan(ch, n_frames);
  const uint32_t nblk =
      __builtin_amdgcn_readfirstlane((wave_max(has ? cp.total : 0u) + kB - 1) / kB);
  // per-lane map parameters, selected without indexing (which would put `ch` in scratch)
  const double p = m ? ch.p[1] : ch.p[0], h = m ? ch.h[1] : ch.h[0];
  const double ip = m ? ch.ip[1] : ch.ip[0], ih = m ? ch.ih[1] : ch.ih[0];
  const double lp = m ? ch.lp[1] : ch.lp[0], lh = m ? ch.lh[1] : ch.lh[0];
  double x = has ? ch.state[m] : 0.0;  // the producer's chain value
  if (wave == 0) ckpt[2][kNV - 1][lane] = x;  // "block -1" ends with the launch's start state
  if (threadIdx.x < 2) fix_count[threadIdx.x] = 0;
  uint32_t hwid;
  asm volatile("s_getreg_b32 %0, hwreg(HW_REG_HW_ID)" : "=s"(hwid));
  if (lane == 0) simd_of[wave] = (hwid >> 4) & 3u;
  uint8_t* base = ks_base + ch.out_off;
  Cursor cu{0, 0};  // emitter lane 2c+q writes steps [16q, 16q+16) of each block
  advance(cu, (lane & 1u) * (kB / 2), cp.spf ? cp.spf : 1);
  uint32_t seen0 = 0, seen1 = 0;  // fix_count values already acted on
  bool repaired = false;          // block b-1 was written by a repair (the same in every wavefront)
  __syncthreads();

  // Roles (the same table in every wavefront): the producer is the first
  // wavefront alone on its SIMD, the emitter the first other one that shares
  // a SIMD (else the first other one), the rest verify, ordered by index
  // except that one sharing the emitter's SIMD comes last.
  uint32_t per_simd = 0;  // 8 bits per SIMD: wavefronts on it
  for (uint32_t w = 0; w < kWaves; w++) per_simd += 1u << (8 * simd_of[w]);
  auto alone = [&](uint32_t w) { return ((per_simd >> (8 * simd_of[w])) & 255u) == 1u; };
  uint32_t prod = kWaves, emit = kWaves;
  for (uint32_t w = 0; w < kWaves; w++)
    if (prod == kWaves && alone(w)) prod = w;
  if (prod == kWaves) prod = 0;
  for (uint32_t w = 0; w < kWaves; w++)
    if (emit == kWaves && w != prod && !alone(w)) emit = w;
  if (emit == kWaves) emit = prod == 0 ? 1 : 0;
  auto vkey = [&](uint32_t w) { return (simd_of[w] == simd_of[emit] ? kWaves : 0u) + w; };
  uint32_t role = wave == prod ? 0u : wave == emit ? 1u : 2u;
  if (role == 2)
    for (uint32_t w = 0; w < kWaves; w++)
      if (w != prod && w != emit && vkey(w) < vkey(wave)) role++;
  role = __builtin_amdgcn_readfirstlane(role);
  __builtin_amdgcn_s_setprio(3);

  for (uint32_t b = 0; b < nblk + 2; b++) {
    if (role == 0) {
      if (b < nblk) {
        double* ck = &ckpt[b % 3][0][lane];
#pragma unroll
        for (uint32_t s = 0; s < kB; s++) {
          x = plcm_two(x, p, ip, lp, ih, lh);
          if constexpr (kPlant)  // testing: a one-bit error in some steps of every lane
            if (planted(b * kB + s, lane, 29))
              x = __longlong_as_double(__double_as_longlong(x) ^ 1);
          if (Seg::ckpt_after(s) < kNV) ck[Seg::ckpt_after(s) * 64] = x;
        }
      }
    } else if (role == 1) {
      if (b >= 2 && has)
        emit_sub<2, kB>(ring[(b - 2) % 3], c, lane & 1u, b - 2, cp, base, ch.frame_stride, cu,
                    ch.state);
    } else if (b >= 1 && b - 1 < nblk && !repaired) {
      // block b-1, unless a repair already wrote it (then its values are exact)
      const uint32_t v = role - 2, blk = b - 1, s0 = v * Seg::kSegLong;
      double* rv = reinterpret_cast<double*>(ring[blk % 3]);
      const double start = v == 0 ? ckpt[(blk + 2) % 3][kNV - 1][lane] : ckpt[blk % 3][v - 1][lane];
      const double end = ckpt[blk % 3][v][lane];  // the producer's checkpoint
      const bool bad =
          v < kNV - 1
              ? verify_segment<Seg::kSegLong, kPlant>(start, end, rv, s0, blk * kB + s0, lane,
                                                      p, h, ip, ih, lp, lh)
              : verify_segment<Seg::kSegLast, kPlant>(start, end, rv, s0, blk * kB + s0, lane,
                                                      p, h, ip, ih, lp, lh);
      // any lane of a chain (lanes past a chain's end hold further orbit
      // values: a failure there costs a repair, never a wrong byte)
      if (__ballot(has && bad) != 0 && lane == 0) atomicAdd(&fix_count[b & 1u], 1u);
    }
    __syncthreads();
    // Counter of this iteration's parity: a wavefront that runs ahead into
    // iteration b+1 adds to the other one, so every wavefront reads the same
    // value here and all or none take the repair branch (and its barrier).
    const uint32_t fc = __builtin_amdgcn_readfirstlane(fix_count[b & 1u]);
    const uint32_t seen = (b & 1u) ? seen1 : seen0;
    repaired = false;
    if (fc != seen) {  // only after a verifier ran (b >= 1)
      if (b & 1u) seen1 = fc; else seen0 = fc;
      if (role == 0) {
        // blocks b-1 and b again from the verified end of block b-2, with
        // the correctly rounded step
        const uint32_t blk = b - 1;
        double y = ckpt[(blk + 2) % 3][kNV - 1][lane];
        for (uint32_t bb = blk; bb <= b && bb < nblk; bb++) {
          double* r = reinterpret_cast<double*>(ring[bb % 3]);
          for (uint32_t s = 0; s < kB; s++) {
            y = plcm_fast(y, p, h, ip, ih);
            r[ring_index(s, lane)] = y;
            if (Seg::ckpt_after(s) < kNV) ckpt[bb % 3][Seg::ckpt_after(s)][lane] = y;
          }
        }
        if (b < nblk) x = y;
      }
      repaired = b < nblk;
      __syncthreads();
    }
  }
}

// Generator states moved between a key and a batch's speculative copy of
// them: workgroup q copies entry q.
__global__ __launch_bounds__(64) void copy_states_kernel(const StateCopy* c, uint32_t n) {
  const StateCopy e = c[blockIdx.x];
  for (uint64_t i = threadIdx.x; i < e.count; i += 64) e.dst[i] = e.src[i];
}

}  // namespace

hipError_t launch_copy_states(const StateCopy* d_copies, uint32_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(copy_states_kernel, dim3(n), dim3(64), 0, s, d_copies, n);
  return hipGetLastError();
}

uint32_t prbg_plcm_workgroups(uint32_t n_chains, int variant) {
  return variant == PRBG_RECIP_PAIR ? (n_chains + 15) / 16 : (n_chains + 31) / 32;
}

hipError_t launch_prbg_plcm(const PlcmChain* d_chains, uint32_t n_chains, uint8_t* ks_base,
                            uint32_t n_frames, int variant, hipStream_t s) {
  if (n_chains == 0) return hipSuccess;
  switch (variant) {
    case PRBG_SPEC:
    case PRBG_SPEC_PLANT: {
      // Up to 64 workgroups (a compute unit each, also on a stream limited
      // to a quarter of the chip): blocks of 64 steps halve the per-block
      // barrier and repair check (103 KB of LDS).  More workgroups: blocks
      // of 32 (54 KB), so that three share a compute unit.
      const bool plant = variant == PRBG_SPEC_PLANT, few = (n_chains + 31) / 32 <= 64;
      const dim3 grid((n_chains + 31) / 32), block((2 + kSpecVerifiers) * 64);
      if (few && !plant)
        hipLaunchKernelGGL((prbg_plcm_spec_kernel<false, kSpecVerifiers, 64>), grid, block, 0, s,
                           d_chains, n_chains, ks_base, n_frames);
      else if (few)
        hipLaunchKernelGGL((prbg_plcm_spec_kernel<true, kSpecVerifiers, 64>), grid, block, 0, s,
                           d_chains, n_chains, ks_base, n_frames);
      else if (!plant)
        hipLaunchKernelGGL((prbg_plcm_spec_kernel<false, kSpecVerifiers, 32>), grid, block, 0, s,
                           d_chains, n_chains, ks_base, n_frames);
      else
        hipLaunchKernelGGL((prbg_plcm_spec_kernel<true, kSpecVerifiers, 32>), grid, block, 0, s,
                           d_chains, n_chains, ks_base, n_frames);
      break;
    }
    case PRBG_RECIP_PAIR:
      hipLaunchKernelGGL(prbg_plcm_kernel<kRecipPair>, dim3((n_chains + 15) / 16), dim3(128), 0, s,
                         d_chains, n_chains, ks_base, n_frames);
      break;
    case PRBG_RECIP:
      hipLaunchKernelGGL(prbg_plcm_kernel<kRecip>, dim3((n_chains + 31) / 32), dim3(128), 0, s,
                         d_chains, n_chains, ks_base, n_frames);
      break;
    default:
      hipLaunchKernelGGL(prbg_plcm_kernel<kExact>, dim3((n_chains + 31) / 32), dim3(128), 0, s,
                         d_chains, n_chains, ks_base, n_frames);
  }
  return hipGetLastError();
}

}  // namespace cv
