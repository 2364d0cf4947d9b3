// Host statistics of probe pressure series: the cumulative RMS vectors of Eqs. (10)-(12), the
// spanwise observer average used for the OASPL of Eq. (9) with several observer points, and the
// Welch power spectral density of the pressure perturbation.  Plain C++ on a few thousand samples
// per probe (FP64); the series come from the FP64 probe accumulator on the device.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <vector>
#include <exception>

#include "../../include/fr.h"

namespace {

// stable running mean / second moment (Welford): element k uses the first k + 1 samples
void cumulative_rms(const double *p, int64_t n, double *out) {
  double mean = 0.0, m2 = 0.0;
  for (int64_t k = 0; k < n; ++k) {
    const double d = p[k] - mean;
    mean += d / (double)(k + 1);
    m2 += d * (p[k] - mean);
    out[k] = std::sqrt(std::max(m2, 0.0) / (double)(k + 1));
  }
}

// one-sided DFT power |sum_t x_t e^{-2 pi i f t / L}|^2 for f = 0 .. L/2 (direct summation with a
// recurrence-free twiddle table; L is a few thousand at most)
void dft_power(const std::vector<double> &x, std::vector<double> &pw) {
  const int64_t L = (int64_t)x.size(), nf = L / 2 + 1;
  std::vector<double> c(L), s(L);
  for (int64_t t = 0; t < L; ++t) {
    const double a = 2.0 * M_PI * (double)t / (double)L;
    c[t] = std::cos(a);
    s[t] = std::sin(a);
  }
  pw.assign(nf, 0.0);
  for (int64_t f = 0; f < nf; ++f) {
    double re = 0.0, im = 0.0;
    int64_t idx = 0;
    for (int64_t t = 0; t < L; ++t) {
      re += x[t] * c[idx];
      im -= x[t] * s[idx];
      idx += f;
      if (idx >= L) idx -= L;
    }
    pw[f] = re * re + im * im;
  }
}

}  // namespace

extern "C" {

fr_status fr_stats_prms_cumulative(const double *series, int64_t n, double *prms) {
  if (!series || !prms || n < 1) return FR_ERR_ARG;
  cumulative_rms(series, n, prms);
  return FR_OK;
}

fr_status fr_stats_observer_oaspl(const double *series, int32_t n_probe, int64_t n, const int32_t *group,
                                  int32_t n_group, double p_ref, double *prms, double *oaspl) {
  if (!series || !group || !prms || !oaspl || n_probe < 1 || n < 1 || n_group < 1 || !(p_ref > 0.0))
    return FR_ERR_ARG;
  try {
    std::vector<double> sum(n_group, 0.0), tmp(n);
    std::vector<int> cnt(n_group, 0);
    for (int32_t a = 0; a < n_probe; ++a) {
      const int32_t g = group[a];
      if (g < 0 || g >= n_group) return FR_ERR_ARG;
      cumulative_rms(series + (int64_t)a * n, n, tmp.data());
      sum[g] += tmp[n - 1];
      cnt[g] += 1;
    }
    for (int32_t g = 0; g < n_group; ++g) {
      if (cnt[g] == 0) return FR_ERR_ARG;
      prms[g] = sum[g] / cnt[g];
      oaspl[g] = prms[g] > 0.0 ? 20.0 * std::log10(prms[g] / p_ref) : -INFINITY;
    }
  } catch (const std::exception &) {  // allocation (bad_alloc, or a size beyond max_size)
    return FR_ERR_OOM;
  }
  return FR_OK;
}

fr_status fr_stats_psd_welch(const double *series, int64_t n, int32_t n_windows, double sample_dt, double *freq,
                             double *psd, int64_t cap, int64_t *n_freq) {
  if (!series || !freq || !psd || !n_freq || n_windows < 1 || !(sample_dt > 0.0)) return FR_ERR_ARG;
  // n_windows segments of even length L overlapping by L/2 cover the first L (n_windows + 1) / 2
  // samples: L = 2 floor(n / (n_windows + 1))
  const int64_t L = 2 * (n / (n_windows + 1));
  if (L < 2) return FR_ERR_ARG;
  const int64_t hop = L / 2, nf = L / 2 + 1;
  *n_freq = nf;
  if (cap < nf) return FR_ERR_ARG;
  std::vector<double> w;
  try {
    w.resize(L);
  } catch (const std::exception &) {  // allocation (bad_alloc, or a size beyond max_size)
    return FR_ERR_OOM;
  }
  double w2 = 0.0;
  for (int64_t t = 0; t < L; ++t) {  // periodic Hann window
    w[t] = 0.5 - 0.5 * std::cos(2.0 * M_PI * (double)t / (double)L);
    w2 += w[t] * w[t];
  }
  const double fs = 1.0 / sample_dt;
  try {
    std::vector<double> acc(nf, 0.0), x(L), pw;
    for (int32_t k = 0; k < n_windows; ++k) {
      const double *seg = series + (int64_t)k * hop;
      double mean = 0.0;
      for (int64_t t = 0; t < L; ++t) mean += seg[t];
      mean /= (double)L;
      for (int64_t t = 0; t < L; ++t) x[t] = (seg[t] - mean) * w[t];  // pressure perturbation per segment
      dft_power(x, pw);
      for (int64_t f = 0; f < nf; ++f) acc[f] += pw[f];
    }
    for (int64_t f = 0; f < nf; ++f) {
      // one-sided density: double every bin except DC and (even L) Nyquist
      const bool edge = f == 0 || (L % 2 == 0 && f == L / 2);
      psd[f] = acc[f] / n_windows / (fs * w2) * (edge ? 1.0 : 2.0);
      freq[f] = (double)f * fs / (double)L;
    }
  } catch (const std::exception &) {  // allocation (bad_alloc, or a size beyond max_size)
    return FR_ERR_OOM;
  }
  return FR_OK;
}

}  // extern "C"
