// cv_apply_rounds_noalloc: the r rounds with a caller-supplied keystream
// (as cv_apply_rounds) for callers that cannot allocate device memory.
//
// Every device buffer the rounds need beyond the caller's frames and
// keystream lives in one file-scope device array of fixed size, `scratch`
// (CV_NOALLOC_SCRATCH_BYTES): the error word and the group-barrier counters
// (header), the frames' shift tables, then either the fused kernels'
// exchange frames (two pixel-word frames per group) or the byte kernels'
// ping-pong frames.  Its device address is looked up once per device with
// hipGetSymbolAddress; host code passes that address, never the symbol.
// The shift tables are staged in a static host array; a copy from pageable
// host memory is synchronous, so the array is free again when it returns.
#include <mutex>

#include "runtime.h"

static __device__ __align__(256) uint8_t scratch[CV_NOALLOC_SCRATCH_BYTES];

namespace cv {
namespace rt {
namespace {

constexpr uint64_t kScratchBytes = CV_NOALLOC_SCRATCH_BYTES;
constexpr uint64_t kCountersOff = 256;     // the error word sits at offset 0
constexpr uint32_t kMaxGroups = 126;       // 128 bytes of counters per group
constexpr uint64_t kHeaderBytes = 16384;   // error word + counters, 256-byte aligned
constexpr uint32_t kStageWords = 1u << 18; // host staging of shift tables (1 MiB)
constexpr int kMaxDevices = 64;
static_assert(kCountersOff + 128ull * kMaxGroups <= kHeaderBytes, "counters overflow the header");

std::mutex g_mu;                        // one call at a time in this process
uint8_t* g_base[kMaxDevices] = {};      // device address of `scratch`, per device
uint32_t g_stage[kStageWords];          // shift tables of one chunk of frames
uint32_t g_err_host;

uint64_t align256(uint64_t x) { return (x + 255) & ~255ull; }

__global__ void clear_word(uint32_t* w) { *w = 0; }

// The device address of `scratch` on the current device (set-up on the
// first call on each device).
cv_status scratch_base(int device, uint8_t** out) {
  if (device < 0 || device >= kMaxDevices) return fail(CV_E_INVAL, "device index too large");
  if (!g_base[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    g_base[device] = (uint8_t*)p;
  }
  *out = g_base[device];
  return CV_OK;
}

}  // namespace
}  // namespace rt
}  // namespace cv

using namespace cv::rt;

extern "C" cv_status cv_apply_rounds_noalloc(cv_key* k, int decrypt, const uint8_t* in,
                                             uint8_t* out, const uint8_t* ks,
                                             const uint32_t* s_c, size_t n, void* stream) {
  cv_status s = check_frames_args(k, in, out, s_c, n);
  if (s != CV_OK || n == 0) return s;
  if (!ks) return fail(CV_E_INVAL, "NULL keystream");
  if ((s = check_async_errors(k, false)) != CV_OK) return s;
  const Geom& g = k->g;
  const uint64_t F = k->F, ks_frame = (uint64_t)g.r * F;
  if (ranges_overlap(ks, n * ks_frame, in, n * F) || ranges_overlap(ks, n * ks_frame, out, n * F))
    return fail(CV_E_INVAL, "keystream overlaps a frame buffer");
  const bool dec = decrypt != 0;
  const bool fused = use_pw(k, in, out, ks) && fused_group_cap(k, dec) > 0;
  const uint64_t tab = (uint64_t)g.H * 4;               // shift table of one frame
  const uint64_t pwf = (uint64_t)g.H * g.W * 4;          // one pixel-word frame
  const uint64_t avail = kScratchBytes - kHeaderBytes;
  // frames per chunk: the staging array, and room for at least one group
  // (fused) or each frame's ping-pong copy (byte kernels)
  uint64_t T = std::min<uint64_t>(n, kStageWords / g.H);
  if (fused) {
    if (2 * pwf + align256(tab) > avail) T = 0;
    else T = std::min<uint64_t>(T, (avail - 2 * pwf - 255) / tab);
  } else {
    T = std::min<uint64_t>(T, (avail - 255) / (F + tab));
  }
  if (T == 0)
    return fail(CV_E_INVAL, "frame too large for the allocation-free scratch (" +
                                std::to_string(kScratchBytes >> 20) + " MiB)");

  std::lock_guard<std::mutex> lock(g_mu);
  DeviceGuard dg(k->device);
  uint8_t* base = nullptr;
  if ((s = scratch_base(k->device, &base)) != CV_OK) return s;
  hipStream_t st = (hipStream_t)stream;
  uint32_t* err = (uint32_t*)base;
  uint32_t* counters = (uint32_t*)(base + kCountersOff);
  uint32_t* gm = (uint32_t*)(base + kHeaderBytes);
  hipLaunchKernelGGL(clear_word, dim3(1), dim3(1), 0, st, err);
  CV_HIP(hipGetLastError());
  for (uint64_t f0 = 0; f0 < n; f0 += T) {
    const uint32_t Tc = (uint32_t)std::min<uint64_t>(T, n - f0);
    for (uint32_t t = 0; t < Tc; t++) shift_table(g.H, g.W, s_c[f0 + t], g_stage + (uint64_t)t * g.H);
    // pageable source: the copy is synchronous, and ordered after the
    // previous chunk's kernels on the stream, which read the same tables
    CV_HIP(hipMemcpyAsync(gm, g_stage, Tc * tab, hipMemcpyHostToDevice, st));
    uint8_t* work = base + kHeaderBytes + align256(Tc * tab);
    const uint8_t* fin = in + f0 * F;
    uint8_t* fout = out + f0 * F;
    const uint8_t* fks = ks + f0 * ks_frame;
    if (fused) {
      const uint64_t room = kScratchBytes - (uint64_t)(work - base);
      const uint32_t groups = (uint32_t)std::min<uint64_t>(kMaxGroups, room / (2 * pwf));
      s = launch_fused_ws(k, dec, fin, fout, fks, Tc, gm, work, counters, err, groups, st);
    } else {
      s = run_rounds_bytes_ws(k, dec, fin, fout, fks, Tc, gm, work, st, false);
    }
    if (s != CV_OK) return s;
    CV_HIP(hipStreamSynchronize(st));
  }
  // pageable destination: synchronous, after the kernels
  CV_HIP(hipMemcpyAsync(&g_err_host, err, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
  CV_HIP(hipStreamSynchronize(st));
  if (g_err_host)
    return fail(CV_E_HIP, "a fused launch timed out at a group barrier or found a group spread "
                          "over XCDs; the output frames of this call are invalid");
  return CV_OK;
}
