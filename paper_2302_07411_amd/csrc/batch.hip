// Many streams in one launch: the r rounds of one tick's frames of many
// video streams with different resolutions and subframe counts (Sec. 2,
// Eq. (1)-(4), Algorithm 1's round loop), on gfx950.
//
// Work is a list of jobs, one per (stream, frame).  A persistent grid is cut
// into groups of G workgroups that share an XCD; a group takes its jobs one
// after the other (the host assigns jobs to groups longest first), and for
// each job and round its workgroup w handles bands w, w+G, w+2G, ... of that
// job's frame -- so streams with 8, 16 or 32 subframes run side by side in
// one grid.  Bands are exchanged through the group's pixel-word scratch with
// the same XCD-local group barrier as the single-stream fused kernel.  Jobs
// must share C (3 or 4); every frame width is a multiple of 16 and every
// buffer 16-byte aligned (the host sends other streams down the per-key
// path).
#include "tile_ops.h"

namespace cv {
namespace {

using namespace tile;

template <uint32_t C>
__global__ __launch_bounds__(kMaxThreads) void batch_rounds_kernel(BatchArgs A) {
  extern __shared__ __align__(16) uint32_t tile_lds[];
  __shared__ uint32_t scan_sh[kMaxThreads / 64];
  const uint32_t i = blockIdx.x, xcd = i % 8, idx = i / 8;
  const uint32_t group = xcd + 8 * (idx / A.G), w = idx % A.G;
  if (group >= A.groups) return;
  uint32_t* ctr = A.counters + 32 * group;
  check_group_xcc(ctr + 1, A.err);
  uint8_t* buf[2] = {A.scratch + (uint64_t)group * 2 * A.scratch_stride,
                     A.scratch + (uint64_t)group * 2 * A.scratch_stride + A.scratch_stride};
  uint32_t nbar = 0;
  for (uint32_t q = A.group_off[group]; q < A.group_off[group + 1]; q++) {
    const BatchJob J = A.jobs[A.group_jobs[q]];
    const Geom g = J.g;
    const uint64_t pwf = (uint64_t)g.H * g.W * 4;
    uint32_t* blo = tile_lds + (size_t)J.tile_rows * g.W;
    uint32_t* seed = blo + g.n + 1;
    View v;
    v.ks = J.ks;
    v.gm = J.gm;
    for (uint32_t s = 0; s < g.r; s++) {
      const bool first = s == 0, last = s + 1 == g.r;
      v.src = first ? J.in : buf[(s + 1) & 1];
      v.src_last = first ? J.in_last : buf[(s + 1) & 1] + pwf - 4;
      v.dst = last ? J.out : buf[s & 1];
      if (!J.decrypt) {
        const uint32_t j = s;
        for (uint32_t band = w; band < g.n; band += A.G) {
          const uint32_t lo = (uint32_t)band_lo(g.H, g.n, band), hi = (uint32_t)band_lo(g.H, g.n, band + 1);
          uint32_t carry = first ? enc_seed<C, true>(v, g, band) : enc_seed<C, false>(v, g, band);
          for (uint32_t t0 = lo; t0 < hi; t0 += J.tile_rows) {
            const uint32_t R = min(J.tile_rows, hi - t0);
            if (first && last) carry = enc_tile<C, true, true>(v, g, j, lo, hi, t0, R, carry, tile_lds, scan_sh);
            else if (first) carry = enc_tile<C, true, false>(v, g, j, lo, hi, t0, R, carry, tile_lds, scan_sh);
            else if (last) carry = enc_tile<C, false, true>(v, g, j, lo, hi, t0, R, carry, tile_lds, scan_sh);
            else carry = enc_tile<C, false, false>(v, g, j, lo, hi, t0, R, carry, tile_lds, scan_sh);
            __syncthreads();
          }
        }
      } else {
        const uint32_t j = g.r - 1 - s;
        if (w < g.n) {
          if (first) dec_seeds<C, true>(v, g, j, blo, seed);
          else dec_seeds<C, false>(v, g, j, blo, seed);
        }
        for (uint32_t band = w; band < g.n; band += A.G) {
          const uint32_t lo = (uint32_t)band_lo(g.H, g.n, band), hi = (uint32_t)band_lo(g.H, g.n, band + 1);
          for (uint32_t t0 = lo; t0 < hi; t0 += J.tile_rows) {
            const uint32_t R = min(J.tile_rows, hi - t0);
            if (first && last) dec_tile<C, true, true>(v, g, j, t0, R, tile_lds, blo, seed);
            else if (first) dec_tile<C, true, false>(v, g, j, t0, R, tile_lds, blo, seed);
            else if (last) dec_tile<C, false, true>(v, g, j, t0, R, tile_lds, blo, seed);
            else dec_tile<C, false, false>(v, g, j, t0, R, tile_lds, blo, seed);
          }
        }
      }
      nbar++;
      if (!group_barrier(ctr, nbar * A.G, A.spin_limit, A.err)) return;
    }
  }
}

__global__ void reset_batch_groups(uint32_t* p, uint32_t groups) {
  for (uint32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < groups; k += gridDim.x * blockDim.x) {
    p[32 * k] = 0;
    p[32 * k + 1] = 0xFFFFFFFFu;
  }
}

}  // namespace

hipError_t launch_batch_rounds(const BatchArgs& a, uint32_t C, uint32_t threads, size_t lds,
                               hipStream_t s) {
  hipLaunchKernelGGL(reset_batch_groups, dim3(1), dim3(256), 0, s, a.counters, a.groups);
  const uint32_t slots = ((a.groups + 7) / 8) * 8 * a.G;
  if (C == 3)
    hipLaunchKernelGGL(batch_rounds_kernel<3>, dim3(slots), dim3(threads), lds, s, a);
  else
    hipLaunchKernelGGL(batch_rounds_kernel<4>, dim3(slots), dim3(threads), lds, s, a);
  return hipGetLastError();
}

uint32_t batch_resident_groups(uint32_t C, uint32_t G, uint32_t threads, size_t lds, int device) {
  int per_cu = 0, cus = 0;
  hipError_t e = C == 3 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, batch_rounds_kernel<3>,
                                                                        threads, lds)
                        : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, batch_rounds_kernel<4>,
                                                                        threads, lds);
  if (e != hipSuccess || per_cu <= 0) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess) return 0;
  const uint32_t per_xcd = (uint32_t)per_cu * (uint32_t)cus / 8;
  return (per_xcd / G) * 8;
}

}  // namespace cv
