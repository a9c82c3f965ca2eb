// fpt_stats.hip -- error bars of the weighted first-passage histogram (Sec. 4.1), computed on
// the host from the histogram accumulators: a few numbers per slot, so no kernel.
//   fpt_jackknife       delete-one jackknife over blocks of trajectories (direct sampling);
//   fpt_lognormal_bins  per-slot lognormal mean of the weights, with Cox's interval and the
//                       count's binomial fluctuation (importance sampling);
//   fpt_merge_bins      inverse-variance merge of runs with different bias amplitudes.
#include "fpt.h"
#include "internal.hpp"

#include <cmath>
#include <vector>

using fpt::report_error;

extern "C" int fpt_jackknife(int32_t n_slots, int32_t n_blocks, const uint64_t *n_traj, const double *sum_w,
                             double *p_out, double *err_out)
{
    if (n_slots < 1) return report_error(FPT_EINVAL, "n_slots must be >= 1");
    if (n_blocks < 2) return report_error(FPT_EINVAL, "the jackknife needs at least 2 blocks");
    if (!n_traj || !sum_w || !p_out || !err_out) return report_error(FPT_EINVAL, "NULL array");
    double N = 0.0;
    for (int b = 0; b < n_blocks; ++b) {
        if (n_traj[b] == 0) return report_error(FPT_EINVAL, "a block has no trajectories");
        N += (double)n_traj[b];
    }
    std::vector<double> loo(n_blocks);
    for (int j = 0; j < n_slots; ++j) {
        double S = 0.0;
        for (int b = 0; b < n_blocks; ++b) {
            const double v = sum_w[(size_t)b * n_slots + j];
            if (!std::isfinite(v)) return report_error(FPT_EINVAL, "non-finite sum_w");
            S += v;
        }
        // estimates with block b left out, and their spread
        double mean = 0.0;
        for (int b = 0; b < n_blocks; ++b) {
            loo[b] = (S - sum_w[(size_t)b * n_slots + j]) / (N - (double)n_traj[b]);
            mean += loo[b];
        }
        mean /= n_blocks;
        double ss = 0.0;
        for (int b = 0; b < n_blocks; ++b) ss += (loo[b] - mean) * (loo[b] - mean);
        p_out[j] = S / N;
        err_out[j] = std::sqrt((double)(n_blocks - 1) / n_blocks * ss);
    }
    return FPT_OK;
}

extern "C" int fpt_lognormal_bins(int32_t n_slots, uint64_t n_traj, const uint64_t *count, const double *sum_lnw,
                                  const double *sum_lnw2, double *p_out, double *lo_out, double *hi_out)
{
    if (n_slots < 1) return report_error(FPT_EINVAL, "n_slots must be >= 1");
    if (n_traj == 0) return report_error(FPT_EINVAL, "n_traj must be >= 1");
    if (!count || !sum_lnw || !sum_lnw2 || !p_out || !lo_out || !hi_out) return report_error(FPT_EINVAL, "NULL array");
    for (int j = 0; j < n_slots; ++j) {
        const double nj = (double)count[j];
        if (count[j] < 2) {
            p_out[j] = lo_out[j] = hi_out[j] = NAN;
            continue;
        }
        // ln w in the slot as N(mu, s^2): mass (n_j/n) e^(mu + s^2/2).  One-sigma half-width of
        // ln(mass): Cox's s^2/n_j + s^4/(2 (n_j - 1)) for ln(mean w), plus the count's binomial
        // (1 - n_j/n)/n_j, in quadrature
        const double mu = sum_lnw[j] / nj;
        const double s2 = std::fmax((sum_lnw2[j] - nj * mu * mu) / (nj - 1.0), 0.0);
        const double theta = mu + 0.5 * s2;
        const double f = nj / (double)n_traj;
        const double se = std::sqrt(s2 / nj + s2 * s2 / (2.0 * (nj - 1.0)) + (1.0 - f) / nj);
        p_out[j] = f * std::exp(theta);
        lo_out[j] = f * std::exp(theta - se);
        hi_out[j] = f * std::exp(theta + se);
    }
    return FPT_OK;
}

extern "C" int fpt_merge_bins(int32_t n_slots, int32_t n_runs, const double *p, const double *err, double *p_out,
                              double *err_out)
{
    if (n_slots < 1 || n_runs < 1) return report_error(FPT_EINVAL, "n_slots and n_runs must be >= 1");
    if (!p || !err || !p_out || !err_out) return report_error(FPT_EINVAL, "NULL array");
    for (int j = 0; j < n_slots; ++j) {
        double sw = 0.0, swp = 0.0;
        for (int r = 0; r < n_runs; ++r) {
            const double v = p[(size_t)r * n_slots + j], e = err[(size_t)r * n_slots + j];
            if (!std::isfinite(v) || !std::isfinite(e) || !(e > 0.0)) continue;   // not usable in this slot
            const double wgt = 1.0 / (e * e);
            sw += wgt;
            swp += wgt * v;
        }
        p_out[j] = sw > 0.0 ? swp / sw : NAN;
        err_out[j] = sw > 0.0 ? 1.0 / std::sqrt(sw) : NAN;
    }
    return FPT_OK;
}
