// Key schedule of the main thread (Algorithm 1): the generator PRBG_m,
// initialised with the key K, is iterated to give the parameters P_m of the
// subframe generators and then, once per frame, a confusion seed s_c.  The
// paper leaves the conversion of iterates into parameters open; this file
// implements reading 1 (CV_KEY_SCHEDULE_VERSION), documented in
// include/chaosvid.h.  PRBG_m is one scalar chain advanced once per frame,
// so it runs on the host (binary64, no contraction; the 2DLASM master uses
// the library's correctly rounded sine).
#include <string.h>

#include <string>

#include "crsin.h"
#include "runtime.h"

using namespace cv::rt;

// The sine tables for host evaluation (key schedule, cv_sin_stage1).
const cv::crsin::LdsTable& cv::rt::crsin_host_table() {
  static const cv::crsin::LdsTable t = [] {
    cv::crsin::LdsTable v;
    for (uint32_t i = 0; i < cv::crsin::kTabEntries; i++) cv::crsin::fill_entry(&v, i);
    return v;
  }();
  return t;
}

namespace {

constexpr int kMaxRejects = 1000;  // consecutive unusable draws before giving up

// Sec. 3, Eq. (5).
double plcm(double x, double p) {
  if (x > 0.5) x = 1.0 - x;
  return x < p ? x / p : (x - p) / (0.5 - p);
}


// One draw (u, v) of PRBG_m: PLCM master -> the new iterates of its two
// maps; 2DLASM master -> the new (x, y) of its map (Eq. 6).
struct Master {
  bool lasm;
  double a, b, c, d;  // PLCM: x1, p1, x2, p2; 2DLASM: x, y, mu
  bool undecided = false;
  void draw(double& u, double& v) {
    if (!lasm) {
      a = plcm(a, b);
      c = plcm(c, d);
      u = a;
      v = c;
      return;
    }
    const double pm = cv::crsin::kPiHi * c;
    const double ax = ((pm * (b + 3.0)) * a) * (1.0 - a);
    const double nx = cv::crsin::cr_sin(ax, &crsin_host_table(), false, &undecided);
    const double ay = ((pm * (nx + 3.0)) * b) * (1.0 - b);
    b = cv::crsin::cr_sin(ay, &crsin_host_table(), false, &undecided);
    a = nx;
    u = a;
    v = b;
  }
  // Next draw whose two values both lie in (0,1).
  bool usable(double& u, double& v) {
    for (int k = 0; k < kMaxRejects; k++) {
      draw(u, v);
      if (u > 0.0 && u < 1.0 && v > 0.0 && v < 1.0) return true;
    }
    return false;
  }
};

bool in_open(double v, double lo, double hi) { return v > lo && v < hi; }

}  // namespace

extern "C" {

cv_status cv_sin_stage1(const double* t, double* hi, double* lo, int* decided, size_t n) {
  if (n && (!t || !hi || !lo || !decided)) return fail(CV_E_INVAL, "NULL argument");
  for (size_t i = 0; i < n; i++)
    if (!(t[i] >= 0.0 && t[i] <= cv::crsin::kPiHi)) return fail(CV_E_INVAL, "t outside [0, RN(pi)]");
  for (size_t i = 0; i < n; i++)
    decided[i] = cv::crsin::sin_quick(t[i], &crsin_host_table(), &hi[i], &lo[i]) ? 1 : 0;
  return CV_OK;
}

cv_status cv_key_schedule(cv_map map, const double* K, size_t n_k, uint32_t n_sub, double* p_m,
                          size_t n_pm, uint64_t first_frame, uint32_t* s_c, size_t n_frames) {
  if (!K || (n_pm && !p_m) || (n_frames && !s_c)) return fail(CV_E_INVAL, "NULL argument");
  if (n_sub == 0) return fail(CV_E_INVAL, "n_sub must be >= 1");
  Master m{};
  if (map == CV_MAP_PLCM) {
    if (n_k != 4) return fail(CV_E_INVAL, "a PLCM master key holds 4 doubles");
    if (!in_open(K[0], 0.0, 1.0) || !in_open(K[2], 0.0, 1.0) || !in_open(K[1], 0.0, 0.5) ||
        !in_open(K[3], 0.0, 0.5))
      return fail(CV_E_INVAL, "PLCM master key: x0 in (0,1), p in (0,1/2)");
    m = Master{false, K[0], K[1], K[2], K[3]};
    if (n_pm != 4ull * n_sub) return fail(CV_E_INVAL, "p_m must hold 4 doubles per subframe");
  } else if (map == CV_MAP_2DLASM) {
    if (n_k != 3) return fail(CV_E_INVAL, "a 2DLASM master key holds 3 doubles (x0, y0, mu)");
    if (!in_open(K[0], 0.0, 1.0) || !in_open(K[1], 0.0, 1.0) || !lasm_mu_ok(K[2]))
      return fail(CV_E_INVAL, "2DLASM master key: x0, y0 in (0,1), mu admissible");
    m = Master{true, K[0], K[1], K[2], 0.0};
    if (n_pm != 6ull * n_sub) return fail(CV_E_INVAL, "p_m must hold 6 doubles per subframe");
  } else {
    return fail(CV_E_INVAL, "unknown map");
  }
  double u = 0, v = 0;
  for (uint32_t i = 0; i < n_sub; i++) {
    if (map == CV_MAP_PLCM) {
      for (int k = 0; k < 2; k++) {
        if (!m.usable(u, v)) return fail(CV_E_INVAL, "degenerate master key");
        p_m[4 * i + 2 * k] = u;
        p_m[4 * i + 2 * k + 1] = v * 0.5;
      }
    } else {
      for (int k = 0; k < 2; k++) {
        if (!m.usable(u, v)) return fail(CV_E_INVAL, "degenerate master key");
        p_m[6 * i + 3 * k] = u;
        p_m[6 * i + 3 * k + 1] = v;
        if (!m.usable(u, v)) return fail(CV_E_INVAL, "degenerate master key");
        p_m[6 * i + 3 * k + 2] = 0.44 + 0.49 * u;
      }
    }
  }
  for (uint64_t t = 0; t < first_frame + n_frames; t++) {
    m.draw(u, v);
    if (t >= first_frame)
      s_c[t - first_frame] =
          1u + (uint32_t)((cv::crsin::bits_of(u) ^ cv::crsin::bits_of(v)) & 0xFFFFu);
  }
  if (m.undecided) return fail(CV_E_HIP, "a 2DLASM sine could not be rounded with certainty");
  return CV_OK;
}

}  // extern "C"
