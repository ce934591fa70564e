// Oscillation diagnostics of a sampled flow functional (Sec. 3.3: the lift
// over the periodic limit cycle; runs are compared after aligning their first
// maximum in the window).  Host code: a few thousand samples per call.
#include <cmath>
#include <cstddef>

#include "dnnmg.h"

extern "C" int dnnmg_oscillation(const double *f, int n, double t0, double dt, double *t_first_max,
                                 double *period, int *n_max) {
  if (!f || n < 3 || !(dt > 0.0) || !std::isfinite(t0)) return DNNMG_EINVAL;
  double mean = 0.0, top = -INFINITY;
  for (int i = 0; i < n; ++i) {
    if (!std::isfinite(f[i])) return DNNMG_EINVAL;
    mean += f[i];
    top = std::fmax(top, f[i]);
  }
  mean /= n;
  const double high = 0.5 * (mean + top);
  // one maximum per excursion above the mean (a maximal run of samples > mean
  // with a sample <= mean on both sides) whose largest sample exceeds the
  // midpoint of mean and global maximum; its time from the parabola through
  // the largest sample and its two neighbours
  int count = 0;
  double first = 0.0, last = 0.0;
  int i = 0;
  while (i < n && f[i] > mean) ++i;   // an excursion cut by the window start is skipped
  while (i < n) {
    while (i < n && !(f[i] > mean)) ++i;
    if (i >= n) break;
    const int b = i;
    int k = i;
    while (i < n && f[i] > mean) {
      if (f[i] > f[k]) k = i;
      ++i;
    }
    if (i >= n) break;                 // cut by the window end
    if (!(f[k] > high) || b == 0) continue;
    const double a = f[k - 1], c = f[k + 1], m = f[k];
    const double curv = a - 2.0 * m + c;
    const double shift = curv < 0.0 ? 0.5 * (a - c) / curv : 0.0;
    const double t = t0 + (k + shift) * dt;
    if (count == 0) first = t;
    last = t;
    ++count;
  }
  if (n_max) *n_max = count;
  if (t_first_max) *t_first_max = count > 0 ? first : NAN;
  if (period) *period = count > 1 ? (last - first) / (count - 1) : NAN;
  return DNNMG_OK;
}
