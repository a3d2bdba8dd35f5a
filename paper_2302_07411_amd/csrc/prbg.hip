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
// latency of one step, not by throughput.  Both maps of a chain run in two
// adjacent lanes of one wavefront (lane 2c: map 1, lane 2c+1: map 2), so a
// step costs the latency of one map; 32 chains share a wavefront for free.
// The pairwise XOR is a DPP lane swap.  Eight steps (48 bytes) are packed in
// registers and written by the even lane as three 16-byte stores.
//
// Every floating-point operation is a single IEEE-754 binary64 operation
// with round-to-nearest-even: built with -ffp-contract=off and no fast-math,
// the division is the compiler's correctly rounded expansion.  A chaotic
// orbit amplifies any rounding difference, so this is what makes the
// keystream bit-identical to any other correct implementation.
#include "cv_internal.h"

namespace cv {
namespace {

// Eq. (5).  x in (1/2,1] is folded to 1-x (exact by Sterbenz' lemma) and
// then mapped by the first two pieces; one division per step.
__device__ __forceinline__ double plcm_step(double x, double p, double h) {
  const double y = (x > 0.5) ? 1.0 - x : x;
  const bool first = y < p;
  const double num = first ? y : y - p;
  const double den = first ? p : h;
  return num / den;
}

// Value of the same register in the adjacent lane (0<->1, 2<->3, ...):
// DPP quad_perm(1,0,3,2).
__device__ __forceinline__ uint32_t swap_pair(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, false);
}

// XOR of this lane's iterate bits with its partner's (both lanes active).
__device__ __forceinline__ uint2 pair_xor_bits(double x) {
  const uint64_t u = (uint64_t)__double_as_longlong(x);
  const uint32_t lo = (uint32_t)u, hi = (uint32_t)(u >> 32);
  return make_uint2(lo ^ swap_pair(lo), hi ^ swap_pair(hi));
}

__global__ __launch_bounds__(64) void prbg_plcm_kernel(const PlcmChain* __restrict__ chains,
                                                        uint32_t n_chains, uint8_t* ks_base,
                                                        uint32_t n_frames) {
  const uint32_t lane = threadIdx.x;
  const uint32_t c = blockIdx.x * 32u + (lane >> 1);
  const uint32_t map = lane & 1u;
  if (c >= n_chains) return;  // both lanes of a pair leave together
  const PlcmChain ch = chains[c];
  const double p = ch.p[map], h = ch.h[map];
  double x = ch.state[map];
  for (uint32_t f = 0; f < n_frames; f++) {
    uint8_t* out = ks_base + ch.out_off + (uint64_t)f * ch.frame_stride;
    uint64_t done = 0;
    if ((((uintptr_t)out) & 15u) == 0) {
      for (; done + 48 <= ch.nbytes; done += 48) {
        uint32_t w[12];
#pragma unroll
        for (int s = 0; s < 4; s++) {
          x = plcm_step(x, p, h);
          const uint2 b0 = pair_xor_bits(x);
          x = plcm_step(x, p, h);
          const uint2 b1 = pair_xor_bits(x);
          // 12 bytes = bytes 0..5 of b0 then bytes 0..5 of b1
          w[3 * s + 0] = b0.x;
          w[3 * s + 1] = (b0.y & 0xFFFFu) | (b1.x << 16);
          w[3 * s + 2] = (b1.x >> 16) | (b1.y << 16);
        }
        if (map == 0) {
          uint4* o4 = reinterpret_cast<uint4*>(out + done);
          o4[0] = make_uint4(w[0], w[1], w[2], w[3]);
          o4[1] = make_uint4(w[4], w[5], w[6], w[7]);
          o4[2] = make_uint4(w[8], w[9], w[10], w[11]);
        }
      }
    }
    // Remaining bytes (and frames whose block is not 16-byte aligned):
    // one step at a time, only the bytes that fit are kept.
    for (; done < ch.nbytes; done += 6) {
      x = plcm_step(x, p, h);
      const uint2 b = pair_xor_bits(x);
      if (map == 0) {
        const uint64_t bits = ((uint64_t)b.y << 32) | b.x;
        const uint64_t left = ch.nbytes - done;
        const int take = left < 6 ? (int)left : 6;
        for (int k = 0; k < take; k++) out[done + k] = (uint8_t)(bits >> (8 * k));
      }
    }
  }
  ch.state[map] = x;
}

}  // namespace

hipError_t launch_prbg_plcm(const PlcmChain* d_chains, uint32_t n_chains, uint8_t* ks_base,
                            uint32_t n_frames, hipStream_t s) {
  if (n_chains == 0 || n_frames == 0) return hipSuccess;
  const uint32_t blocks = (n_chains + 31) / 32;
  hipLaunchKernelGGL(prbg_plcm_kernel, dim3(blocks), dim3(64), 0, s, d_chains, n_chains, ks_base,
                     n_frames);
  return hipGetLastError();
}

}  // namespace cv
