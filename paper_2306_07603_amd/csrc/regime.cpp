// regime.cpp -- host-side spectral classification of a probe time series
// (the steady / periodic / quasi-periodic regimes of Section 6.2 of
// arXiv:2306.07603, read from the velocity at the cavity centre or the
// kinetic energy of Eq. (5.1)).
//
// Method: a relative fluctuation amplitude at or below the tolerance is a
// steady state.  Otherwise remove the least-squares line (mean and drift),
// Hann-window the series, zero-pad it to a power of two at least four times its
// length, take the power spectrum with an iterative radix-2 Cooley-Tukey FFT,
// and locate the strongest spectral peak above 1.5 cycles per record: a bin
// that is a local maximum (frequency refined by a parabola through the
// logarithms of the three bins around it).  The share of the whole
// fluctuation energy within the main lobe of the peak frequency and of its
// integer multiples decides "periodic"; otherwise a second narrow peak away
// from those multiples that holds most of the rest decides "quasi-periodic";
// anything else is "aperiodic".  A series still relaxing (a drift that is not
// a straight line, or a period longer than the record) keeps most of its
// energy below 1.5 cycles per record and is therefore "aperiodic".
#include "ifdlbm.h"

#include <algorithm>
#include <cmath>
#include <complex>
#include <new>
#include <string>
#include <vector>

namespace ifd {
int fail(int code, const std::string& msg);
}

namespace {

// Periodic: this share of the fluctuation energy at the principal frequency and its multiples.
constexpr double kPeriodicShare = 0.9;
// Quasi-periodic: a second peak holding this share of the energy and at least
// half of what the multiples of the principal frequency leave.
constexpr double kSecondShare = 0.02;
constexpr int kPad = 4;   // zero padding factor

void fft(std::vector<std::complex<double>>& a)
{
    const size_t n = a.size();
    for (size_t i = 1, j = 0; i < n; ++i) {   // bit-reversal permutation
        size_t bit = n >> 1;
        for (; j & bit; bit >>= 1) j ^= bit;
        j ^= bit;
        if (i < j) std::swap(a[i], a[j]);
    }
    for (size_t len = 2; len <= n; len <<= 1) {
        const double ang = -2.0 * M_PI / (double)len;
        for (size_t i = 0; i < n; i += len)
            for (size_t k = 0; k < len / 2; ++k) {
                const std::complex<double> w(std::cos(ang * (double)k), std::sin(ang * (double)k));
                const std::complex<double> u = a[i + k], v = a[i + k + len / 2] * w;
                a[i + k] = u + v;
                a[i + k + len / 2] = u - v;
            }
    }
}

// Peak bin refined by a parabola through ln P at k-1, k, k+1.
double refine(const std::vector<double>& P, size_t k)
{
    if (k == 0 || k + 1 >= P.size() || P[k - 1] <= 0 || P[k + 1] <= 0 || P[k] <= 0) return (double)k;
    const double a = std::log(P[k - 1]), b = std::log(P[k]), c = std::log(P[k + 1]);
    const double den = a - 2 * b + c;
    if (den >= 0) return (double)k;
    return (double)k + 0.5 * (a - c) / den;
}

}  // namespace

namespace {

int classify(const double* x, int64_t n, double dt_sample, double steady_tol, ifdlbm_regime_t* out)
{
    using ifd::fail;
    if (!x || !out) return fail(IFDLBM_EINVAL, "null series or output");
    if (n < 16) return fail(IFDLBM_EINVAL, "need at least 16 samples");
    if (n > ((int64_t)1 << 22)) return fail(IFDLBM_EINVAL, "at most 2^22 samples");
    if (!(dt_sample > 0.0) || !(steady_tol >= 0.0)) return fail(IFDLBM_EINVAL, "dt_sample must be > 0, steady_tol >= 0");
    for (int64_t i = 0; i < n; ++i)
        if (!std::isfinite(x[i])) return fail(IFDLBM_EINVAL, "series holds a non-finite value");
    ifdlbm_regime_t r{};
    double mean = 0.0, lo = x[0], hi = x[0], peak = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        mean += x[i];
        lo = std::min(lo, x[i]);
        hi = std::max(hi, x[i]);
        peak = std::max(peak, std::fabs(x[i]));
    }
    mean /= (double)n;
    r.mean = mean;
    r.rel_amplitude = peak > 0.0 ? 0.5 * (hi - lo) / peak : 0.0;
    if (r.rel_amplitude <= steady_tol) {
        r.regime = IFDLBM_REGIME_STEADY;
        *out = r;
        return IFDLBM_OK;
    }
    // least-squares line through the series, about its centre
    const double tc = 0.5 * (double)(n - 1);
    double stx = 0.0, stt = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        stx += ((double)i - tc) * (x[i] - mean);
        stt += ((double)i - tc) * ((double)i - tc);
    }
    const double slope = stx / stt;
    size_t N = 1;
    while (N < (size_t)n * kPad) N <<= 1;
    std::vector<std::complex<double>> a(N, 0.0);
    for (int64_t i = 0; i < n; ++i) {
        const double w = 0.5 - 0.5 * std::cos(2.0 * M_PI * (double)i / (double)(n - 1));
        a[(size_t)i] = (x[i] - mean - slope * ((double)i - tc)) * w;
    }
    fft(a);
    std::vector<double> P(N / 2 + 1);
    for (size_t k = 0; k <= N / 2; ++k) P[k] = std::norm(a[k]);
    // bins below 1.5 cycles per record carry the window's leakage of the mean and trends
    const size_t k_lo = (size_t)std::ceil(1.5 * (double)N / (double)n);
    const double lobe = 2.0 * (double)N / (double)n;   // Hann main-lobe half width, in bins
    // shares are taken of the whole fluctuation spectrum, so that energy below
    // 1.5 cycles per record (an unfinished transient) counts against a peak
    double total = 0.0;
    for (size_t k = 1; k < P.size(); ++k) total += P[k];
    size_t k1 = 0;   // strongest local maximum strictly above k_lo
    for (size_t k = k_lo + 1; k + 1 < P.size(); ++k)
        if (P[k] >= P[k - 1] && P[k] >= P[k + 1] && (k1 == 0 || P[k] > P[k1])) k1 = k;
    if (!(total > 0.0) || k_lo >= P.size() || k1 == 0) {
        r.regime = IFDLBM_REGIME_APERIODIC;
        *out = r;
        return IFDLBM_OK;
    }
    const double kf = refine(P, k1);
    r.f_main = kf / ((double)N * dt_sample);
    std::vector<char> harmonic(P.size(), 0);
    double e_h = 0.0;
    for (int m = 1; m * kf - lobe < (double)(P.size() - 1); ++m) {
        const double c = m * kf;
        const size_t b0 = (size_t)std::max((double)k_lo, std::ceil(c - lobe));
        const size_t b1 = (size_t)std::min((double)(P.size() - 1), std::floor(c + lobe));
        for (size_t k = b0; k <= b1; ++k)
            if (!harmonic[k]) {
                harmonic[k] = 1;
                e_h += P[k];
            }
    }
    r.harmonic_fraction = e_h / total;
    size_t k2 = 0;
    for (size_t k = k_lo; k < P.size(); ++k)
        if (!harmonic[k] && (k2 == 0 || P[k] > P[k2])) k2 = k;
    if (k2) {
        const double kf2 = refine(P, k2);
        r.f_second = kf2 / ((double)N * dt_sample);
        double e2 = 0.0;
        for (size_t k = (size_t)std::max((double)k_lo, std::ceil(kf2 - lobe));
             k <= (size_t)std::min((double)(P.size() - 1), std::floor(kf2 + lobe)); ++k)
            if (!harmonic[k]) e2 += P[k];
        r.second_fraction = e2 / total;
    }
    if (r.harmonic_fraction >= kPeriodicShare)
        r.regime = IFDLBM_REGIME_PERIODIC;
    else if (r.second_fraction >= kSecondShare && r.second_fraction >= 0.5 * (1.0 - r.harmonic_fraction))
        r.regime = IFDLBM_REGIME_QUASI_PERIODIC;
    else
        r.regime = IFDLBM_REGIME_APERIODIC;
    *out = r;
    return IFDLBM_OK;
}

}  // namespace

extern "C" int ifdlbm_classify(const double* x, int64_t n, double dt_sample, double steady_tol, ifdlbm_regime_t* out)
{
    try {
        return classify(x, n, dt_sample, steady_tol, out);
    } catch (const std::bad_alloc&) {
        return ifd::fail(IFDLBM_ENOMEM, "host memory allocation failed");
    } catch (...) {
        return ifd::fail(IFDLBM_EDEVICE, "unexpected C++ exception in the library");
    }
}
