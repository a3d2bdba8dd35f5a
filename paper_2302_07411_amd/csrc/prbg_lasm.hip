// 2DLASM keystream generator (Sec. 3, Eq. (6)) for gfx950.
//
// Every band owns two 2D logistic-adjusted-sine maps; one step of a map is
//   x' = sin(pi*mu*(y+3)*x*(1-x)),  then  y' = sin(pi*mu*(x'+3)*y*(1-y)),
// products in binary64 from left to right (pi = RN(pi)) and the sine
// correctly rounded, so every bit of every iterate is defined.  Each step
// yields 12 keystream bytes: bytes 0..5 of x'(map 1) XOR x'(map 2), then
// bytes 0..5 of y'(map 1) XOR y'(map 2); a band takes ceil(r*S_i/12) steps
// per frame and drops the unused bytes of the last one.  The map state
// persists across frames and calls.
//
// Workgroup: wavefront 0 iterates the maps (lane 2c + m: chain c, map m;
// 32 chains), wavefront 1 turns the iterates of the previous block into
// bytes; an LDS ring of two blocks of kB steps sits between them.
#include "crsin.h"
#include "cv_internal.h"

namespace cv {
namespace {

constexpr uint32_t kB = 16;  // steps per ring block

struct LasmPlan {
  uint64_t nbytes;
  uint32_t spf, total;
};

__device__ __forceinline__ LasmPlan lasm_plan(const LasmChain& ch, uint32_t n_frames) {
  LasmPlan p;
  p.nbytes = ch.nbytes;
  p.spf = (uint32_t)((ch.nbytes + 11) / 12);
  p.total = p.spf * (n_frames ? n_frames : ch.frames);
  return p;
}

__global__ __launch_bounds__(128) void prbg_lasm_kernel(const LasmChain* __restrict__ chains,
                                                        uint32_t n_chains, uint8_t* ks_base,
                                                        uint32_t n_frames, uint32_t force_exact,
                                                        uint32_t* err) {
  __shared__ double2 ring[2][kB][64];
  __shared__ crsin::LdsTable tab;
  crsin::stage_table(&tab);
  __syncthreads();
  const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
  const uint32_t c0 = blockIdx.x * 32;
  const uint32_t nch = min(32u, n_chains - c0);
  const uint32_t c = lane >> 1;
  const bool has = c < nch;
  LasmChain ch{};
  if (has) ch = chains[c0 + c];
  const LasmPlan cp = lasm_plan(ch, n_frames);
  uint32_t tmax = has ? cp.total : 0u;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) tmax = max(tmax, (uint32_t)__shfl_xor((int)tmax, d, 64));
  const uint32_t nblk = (tmax + kB - 1) / kB;
  __builtin_amdgcn_s_setprio(3);  // a latency-bound chain: issue ahead of throughput work

  if (wave == 0) {
    const uint32_t m = lane & 1u;
    double x = has ? ch.state[2 * m] : 0.0, y = has ? ch.state[2 * m + 1] : 0.0;
    const double pm = crsin::kPiHi * ch.mu[m];  // pi*mu, the first product of Eq. (6)
    bool undecided = false;
    for (uint32_t b = 0; b < nblk; b++) {
      for (uint32_t s = 0; s < kB; s++) {
        const double ax = ((pm * (y + 3.0)) * x) * (1.0 - x);
        const double nx = crsin::cr_sin(ax, &tab, force_exact != 0, &undecided);
        const double ay = ((pm * (nx + 3.0)) * y) * (1.0 - y);
        y = crsin::cr_sin(ay, &tab, force_exact != 0, &undecided);
        x = nx;
        ring[b & 1u][s][lane] = make_double2(x, y);
      }
      __syncthreads();
    }
    if (undecided && has) __hip_atomic_store(err, 2u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  } else {
    const uint32_t q = lane & 1u;  // consumer lane q of chain c: steps [q*kB/2, (q+1)*kB/2)
    uint8_t* base = ks_base + ch.out_off;
    // bytes of ring block `blk` (the producer filled it before the last barrier)
    auto emit = [&](uint32_t blk) {
      for (uint32_t s = q * (kB / 2); s < (q + 1) * (kB / 2); s++) {
        const uint32_t g = blk * kB + s;
        if (g >= cp.total) break;
        const double2 a = ring[blk & 1u][s][2 * c], e = ring[blk & 1u][s][2 * c + 1];
        if (g + 1 == cp.total) {  // the chain's state after this launch
          ch.state[0] = a.x;
          ch.state[1] = a.y;
          ch.state[2] = e.x;
          ch.state[3] = e.y;
        }
        const uint64_t X = (uint64_t)__double_as_longlong(a.x) ^ (uint64_t)__double_as_longlong(e.x);
        const uint64_t Y = (uint64_t)__double_as_longlong(a.y) ^ (uint64_t)__double_as_longlong(e.y);
        const uint32_t f = g / cp.spf, sf = g - f * cp.spf;
        const uint64_t at = (uint64_t)sf * 12;
        const uint64_t left = cp.nbytes - at;
        const int take = left < 12 ? (int)left : 12;
        uint8_t* o = base + (uint64_t)f * ch.frame_stride + at;
        for (int k = 0; k < take; k++) o[k] = (uint8_t)(k < 6 ? X >> (8 * k) : Y >> (8 * (k - 6)));
      }
    };
    for (uint32_t b = 0; b < nblk; b++) {
      if (b > 0 && has) emit(b - 1);
      __syncthreads();
    }
    if (nblk > 0 && has) emit(nblk - 1);  // the last block, after the producer's last barrier
  }
}

__global__ void cr_sin_kernel(const double* __restrict__ t, double* __restrict__ out, uint64_t n,
                              uint32_t force_exact, uint32_t* undecided) {
  __shared__ crsin::LdsTable tab;
  crsin::stage_table(&tab);
  __syncthreads();
  bool und = false;
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x)
    out[i] = crsin::cr_sin(t[i], &tab, force_exact != 0, &und);
  if (und) __hip_atomic_store(undecided, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

}  // namespace

hipError_t launch_prbg_lasm(const LasmChain* d_chains, uint32_t n_chains, uint8_t* ks_base,
                            uint32_t n_frames, uint32_t force_exact, uint32_t* err, hipStream_t s) {
  if (n_chains == 0) return hipSuccess;
  hipLaunchKernelGGL(prbg_lasm_kernel, dim3((n_chains + 31) / 32), dim3(128), 0, s, d_chains,
                     n_chains, ks_base, n_frames, force_exact, err);
  return hipGetLastError();
}

hipError_t launch_cr_sin(const double* t, double* out, uint64_t n, uint32_t force_exact,
                         uint32_t* undecided, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const uint64_t blocks = std::min<uint64_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(cr_sin_kernel, dim3((uint32_t)blocks), dim3(256), 0, s, t, out, n, force_exact,
                     undecided);
  return hipGetLastError();
}

}  // namespace cv
