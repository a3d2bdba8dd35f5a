// Many streams in one launch: the r rounds of one tick's frames of many
// video streams with different resolutions and subframe counts (Sec. 2,
// Eq. (1)-(4), Algorithm 1's round loop), on gfx950.
//
// Work is a list of jobs, one per (stream, frame).  A persistent grid is cut
// into groups of workgroups that share an XCD (a table gives each workgroup
// its group, its index w in it and the group's size G; sizes may differ, so
// that a frame with many subframes can get a larger group); a group takes
// its jobs one after the other (the host assigns jobs to groups longest
// first), and for each job and round its workgroup w handles bands w, w+G,
// w+2G, ... of that job's frame -- so streams with 8, 16 or 32 subframes run
// side by side in one grid.  Bands are exchanged through the group's pixel-word scratch with
// the same XCD-local group barrier as the single-stream fused kernel.  Jobs
// must share C (3 or 4); every frame width is a multiple of 16 and every
// buffer 16-byte aligned (the host sends other streams down the per-key
// path).
//
// Two kernels: the pixel-word one (any workgroup size), and the row-run one
// (1024 threads): encryption by whole
// source-row runs with packed-byte diffusion, decryption in one pass per
// tile reading the round input, its predecessors and keystream as
// contiguous runs (skew_ops.h).
#include "skew_ops.h"

namespace cv {
namespace {

using namespace tile;

template <uint32_t C>
__global__ __launch_bounds__(kMaxThreads) void batch_rounds_kernel(BatchArgs A) {
  extern __shared__ __align__(16) uint32_t tile_lds[];
  __shared__ uint32_t scan_sh[kMaxThreads / 64];
  const uint32_t sl = A.slots[blockIdx.x];
  if (sl == kIdleSlot) return;
  const uint32_t group = sl & 0xFFFu, w = (sl >> 12) & 0x3FFu, G = sl >> 22;
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
        for (uint32_t band = w; band < g.n; band += G) {
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
        for (uint32_t band = w; band < g.n; band += G) {
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
      if (!group_barrier(ctr, nbar * G, A.spin_limit, A.err)) return;
    }
  }
}

// One encryption tile of the row-run kernel with the variant's flags (runs
// of 12 pixels per lane when W is a multiple of 12, else of 4).
template <uint32_t C, uint32_t KQ, bool kFull>
__device__ __forceinline__ uint32_t enc_rows_tile(bool first, bool last, const View& v,
                                                  const Geom& g, uint32_t j, uint32_t lo,
                                                  uint32_t hi, uint32_t t0, uint32_t R,
                                                  uint32_t carry, int64_t sa, uint32_t* lds,
                                                  uint32_t* wsum) {
  using skew::skew_tile;
  if (first && last) return skew_tile<C, KQ, true, true, kFull>(v, g, j, lo, hi, t0, R, carry, sa, lds, wsum);
  if (first) return skew_tile<C, KQ, true, false, kFull>(v, g, j, lo, hi, t0, R, carry, sa, lds, wsum);
  if (last) return skew_tile<C, KQ, false, true, kFull>(v, g, j, lo, hi, t0, R, carry, sa, lds, wsum);
  return skew_tile<C, KQ, false, false, kFull>(v, g, j, lo, hi, t0, R, carry, sa, lds, wsum);
}

// Rows [t0, t0+R) of the tile (row pitch W+4) to the round output: packed
// bytes (last round) or pixel words, 4 pixels per lane.
template <uint32_t C>
__device__ __forceinline__ void store_rows(const uint32_t* tile, uint32_t W, uint32_t t0,
                                           uint32_t R, uint8_t* dst, bool packed) {
  const uint32_t pitch = W + 4;
  for (uint32_t q = threadIdx.x; q < R * W / 4; q += blockDim.x) {
    const uint32_t k = (4 * q) / W, c = 4 * q - k * W;
    const uint4 y = *reinterpret_cast<const uint4*>(tile + k * pitch + c);
    if (!packed) {
      gstore4(dst + 4ull * ((uint64_t)t0 * W + 4 * q), y);
    } else if constexpr (C == 4) {
      gstore4(dst + 4ull * ((uint64_t)t0 * W + 4 * q), y);
    } else {
      const uint32_t w4[4] = {y.x, y.y, y.z, y.w};
      uint32_t P[3];
      pack4(w4, P);
      gu32* o = (gu32*)(dst + 3ull * ((uint64_t)t0 * W + 4 * q));
      o[0] = P[0];
      o[1] = P[1];
      o[2] = P[2];
    }
  }
}

template <uint32_t C, uint32_t KQ>
__global__ __launch_bounds__(skew::kThreads) void batch_rows_kernel(BatchArgs A) {
  extern __shared__ __align__(16) uint32_t lds[];
  __shared__ uint32_t wsum[skew::kWaves];
  const uint32_t sl = A.slots[blockIdx.x];
  if (sl == kIdleSlot) return;
  const uint32_t group = sl & 0xFFFu, w = (sl >> 12) & 0x3FFu, G = sl >> 22;
  uint32_t* ctr = A.counters + 32 * group;
  check_group_xcc(ctr + 1, A.err);
  uint8_t* buf[2] = {A.scratch + (uint64_t)group * 2 * A.scratch_stride,
                     A.scratch + (uint64_t)group * 2 * A.scratch_stride + A.scratch_stride};
  uint32_t nbar = 0;
  for (uint32_t q = A.group_off[group]; q < A.group_off[group + 1]; q++) {
    const BatchJob J = A.jobs[A.group_jobs[q]];
    const Geom g = J.g;
    const uint64_t pwf = (uint64_t)g.H * g.W * 4;
    const bool full = g.W % g.H == 0;
    View v;
    v.ks = J.ks;
    v.gm = J.gm;
    uint32_t* gsh = lds + J.tile_dec * (g.W + 4);  // decryption: shift table, bands, seeds
    uint32_t* blo = gsh + g.H;
    uint32_t* seed = blo + g.n + 1;
    if (J.decrypt) {
      __syncthreads();  // the previous job's last reads of the LDS are done
      for (uint32_t a = threadIdx.x; a < g.H; a += blockDim.x) gsh[a] = J.gm[a];
      __syncthreads();
    }
    for (uint32_t s = 0; s < g.r; s++) {
      const bool first = s == 0, last = s + 1 == g.r;
      v.src = first ? J.in : buf[(s + 1) & 1];
      v.src_last = first ? J.in_last : buf[(s + 1) & 1] + pwf - 4;
      v.dst = last ? J.out : buf[s & 1];
      if (!J.decrypt) {
        for (uint32_t band = w; band < g.n; band += G) {
          const uint32_t lo = (uint32_t)band_lo(g.H, g.n, band), hi = (uint32_t)band_lo(g.H, g.n, band + 1);
          const int64_t seed_at = (int64_t)enc_seed_index(v, g, band);
          uint32_t carry = 0;
          for (uint32_t t0 = lo; t0 < hi; t0 += J.tile_enc) {
            const uint32_t R = min(J.tile_enc, hi - t0);
            const int64_t sa = t0 == lo ? seed_at : -1;
            // KQ = 0: runs of 12 or of 4 pixels, by the job's width
            constexpr uint32_t kq12 = KQ == 0 ? 12u : KQ, kq4 = KQ == 0 ? 4u : KQ;
            if (KQ == 0 ? g.W % 12 == 0 : true)
              carry = full ? enc_rows_tile<C, kq12, true>(first, last, v, g, s, lo, hi, t0, R, carry, sa, lds, wsum)
                           : enc_rows_tile<C, kq12, false>(first, last, v, g, s, lo, hi, t0, R, carry, sa, lds, wsum);
            else
              carry = full ? enc_rows_tile<C, kq4, true>(first, last, v, g, s, lo, hi, t0, R, carry, sa, lds, wsum)
                           : enc_rows_tile<C, kq4, false>(first, last, v, g, s, lo, hi, t0, R, carry, sa, lds, wsum);
            __syncthreads();  // the next tile's gather overwrites the LDS tile and wsum
          }
        }
      } else {
        const uint32_t j = g.r - 1 - s;
        if (first) dec_seeds<C, true>(v, g, j, blo, seed);
        else dec_seeds<C, false>(v, g, j, blo, seed);
        for (uint32_t band = w; band < g.n; band += G) {
          const uint32_t lo = blo[band], hi = blo[band + 1];
          for (uint32_t t0 = lo; t0 < hi; t0 += J.tile_dec) {
            const uint32_t R = min(J.tile_dec, hi - t0);
            if (first) {
              if (full) skew::unskew_rows<C, true, true>(v, g, j, t0, R, gsh, blo, seed, lds);
              else skew::unskew_rows<C, true, false>(v, g, j, t0, R, gsh, blo, seed, lds);
            } else {
              if (full) skew::unskew_rows<C, false, true>(v, g, j, t0, R, gsh, blo, seed, lds);
              else skew::unskew_rows<C, false, false>(v, g, j, t0, R, gsh, blo, seed, lds);
            }
            __syncthreads();
            store_rows<C>(lds, g.W, t0, R, v.dst, last);
            __syncthreads();  // the next tile's pass overwrites the tile
          }
        }
      }
      nbar++;
      if (!group_barrier(ctr, nbar * G, A.spin_limit, A.err)) return;
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

static const void* rows_fn(uint32_t C, uint32_t KQ) {
  if (KQ == 0) return C == 3 ? reinterpret_cast<const void*>(&batch_rows_kernel<3, 0>)
                             : reinterpret_cast<const void*>(&batch_rows_kernel<4, 0>);
  if (C == 3) return KQ == 12 ? reinterpret_cast<const void*>(&batch_rows_kernel<3, 12>)
                              : reinterpret_cast<const void*>(&batch_rows_kernel<3, 4>);
  return KQ == 12 ? reinterpret_cast<const void*>(&batch_rows_kernel<4, 12>)
                  : reinterpret_cast<const void*>(&batch_rows_kernel<4, 4>);
}

hipError_t launch_batch_rounds(const BatchArgs& a, uint32_t C, uint32_t KQ, bool rows,
                               uint32_t threads, size_t lds, hipStream_t s) {
  hipLaunchKernelGGL(reset_batch_groups, dim3(1), dim3(256), 0, s, a.counters, a.groups);
  const uint32_t slots = a.n_slots;
  if (rows) {
    const void* fn = rows_fn(C, KQ);
    if (lds > 64 * 1024) {
      const hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (e != hipSuccess) return e;
    }
    BatchArgs copy = a;
    void* args[] = {&copy};
    return hipLaunchKernel(fn, dim3(slots), dim3(skew::kThreads), args, lds, s);
  }
  if (C == 3)
    hipLaunchKernelGGL(batch_rounds_kernel<3>, dim3(slots), dim3(threads), lds, s, a);
  else
    hipLaunchKernelGGL(batch_rounds_kernel<4>, dim3(slots), dim3(threads), lds, s, a);
  return hipGetLastError();
}

namespace {

size_t align256(size_t v) { return (v + 255) / 256 * 256; }

__global__ void fill_stream_rows(BatchJob* jobs, uint32_t* group_jobs, uint32_t* group_off,
                                 uint32_t* slots, BatchJob proto, uint64_t F, uint64_t ks_stride,
                                 uint32_t T, uint32_t groups, uint32_t G, uint32_t n_slots) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t per = T / groups, rem = T % groups;  // groups below rem take per + 1 frames
  if (i < T) {
    BatchJob J = proto;
    J.in += i * F;
    J.out += i * F;
    J.ks += i * ks_stride;
    J.gm += (uint64_t)i * proto.g.H;
    jobs[i] = J;
    const uint32_t q = i % groups, m = i / groups;
    group_jobs[q * per + min(q, rem) + m] = i;
  }
  if (i <= groups) group_off[i] = i * per + min(i, rem);
  if (i < n_slots) {
    const uint32_t xcd = i % 8, u = i / 8, group = xcd + 8 * (u / G);
    slots[i] = group < groups ? batch_slot(group, u % G, G) : kIdleSlot;
  }
}

struct StreamRowsLayout {
  size_t jobs, group_jobs, group_off, slots, bytes;
};

StreamRowsLayout stream_rows_layout(uint32_t T, uint32_t n_slots) {
  StreamRowsLayout L;
  L.jobs = 0;
  L.group_jobs = align256((size_t)T * sizeof(BatchJob));
  L.group_off = L.group_jobs + align256(4 * (size_t)T);
  L.slots = L.group_off + align256(4 * ((size_t)T + 1));
  L.bytes = L.slots + 4 * (size_t)n_slots;
  return L;
}

}  // namespace

size_t stream_rows_table_bytes(uint32_t T, uint32_t n_slots) {
  return stream_rows_layout(T, n_slots).bytes;
}

uint32_t stream_rows_slots(uint32_t groups, uint32_t G) { return 8 * ((groups + 7) / 8) * G; }

hipError_t launch_stream_rows(const StreamRows& s, hipStream_t st) {
  if (s.T == 0 || s.groups == 0 || s.G == 0) return hipErrorInvalidValue;
  const uint32_t groups = min(s.groups, s.T);  // no group without a frame
  const uint32_t n_slots = stream_rows_slots(groups, s.G);
  const StreamRowsLayout L = stream_rows_layout(s.T, n_slots);
  BatchJob* jobs = reinterpret_cast<BatchJob*>(s.tables + L.jobs);
  uint32_t* group_jobs = reinterpret_cast<uint32_t*>(s.tables + L.group_jobs);
  uint32_t* group_off = reinterpret_cast<uint32_t*>(s.tables + L.group_off);
  uint32_t* slots = reinterpret_cast<uint32_t*>(s.tables + L.slots);
  const Geom& g = s.proto.g;
  const uint64_t F = (uint64_t)g.H * g.W * g.C;
  const uint32_t cover = max(s.T + 1, n_slots);
  hipLaunchKernelGGL(fill_stream_rows, dim3((cover + 255) / 256), dim3(256), 0, st, jobs, group_jobs,
                     group_off, slots, s.proto, F, s.ks_stride, s.T, groups, s.G, n_slots);
  BatchArgs a{};
  a.jobs = jobs;
  a.group_jobs = group_jobs;
  a.group_off = group_off;
  a.slots = slots;
  a.scratch = s.scratch;
  a.scratch_stride = (uint64_t)g.H * g.W * 4;
  a.counters = s.counters;
  a.err = s.err;
  a.n_slots = n_slots;
  a.groups = groups;
  a.spin_limit = s.spin_limit;
  return launch_batch_rounds(a, g.C, s.KQ, true, skew::kThreads, s.lds, st);
}

uint32_t batch_resident_slots(uint32_t C, uint32_t KQ, bool rows, uint32_t threads, size_t lds,
                              int device, uint32_t reserve_cus, uint32_t min_wgs) {
  int per_cu = 0, cus = 0;
  hipError_t e;
  if (rows) {
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, rows_fn(C, KQ), skew::kThreads, lds);
  } else {
    e = C == 3 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, batch_rounds_kernel<3>, threads, lds)
               : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, batch_rounds_kernel<4>, threads, lds);
  }
  if (e != hipSuccess || per_cu <= 0) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess) return 0;
  const uint32_t cus_xcd = (uint32_t)cus / 8;
  uint32_t per_xcd = (uint32_t)per_cu * (cus_xcd > reserve_cus ? cus_xcd - reserve_cus : 0);
  if (per_xcd < min_wgs) per_xcd = (uint32_t)per_cu * cus_xcd;
  return per_xcd;
}

size_t batch_rows_lds_bytes(const Geom& g, bool decrypt, uint32_t tile_rows) {
  if (!decrypt) return rounds_skew_lds_bytes(g, tile_rows);
  return ((size_t)tile_rows * (g.W + 4) + g.H + 2 * (size_t)g.n + 2) * 4;
}

uint32_t batch_unskew_tile_rows(const Geom& g, size_t lds_max) {
  if (!((g.C == 3 || g.C == 4) && g.W % 16 == 0)) return 0;
  const size_t reserve = 1024;  // static LDS of the kernel and group-barrier words
  const size_t fixed = ((size_t)g.H + 2 * (size_t)g.n + 2) * 4 + reserve;
  if (lds_max <= fixed) return 0;
  uint32_t rows = (uint32_t)((lds_max - fixed) / ((size_t)(g.W + 4) * 4));
  uint32_t band_max = 0;
  for (uint32_t i = 0; i < g.n; i++)
    band_max = std::max<uint32_t>(band_max, (uint32_t)(band_lo(g.H, g.n, i + 1) - band_lo(g.H, g.n, i)));
  rows = std::min(rows, band_max);
  const uint32_t M = (g.W + g.H - 1) / g.H;
  rows = std::min(rows, skew::kThreads / M);
  return rows;
}

}  // namespace cv
