// fpt_stats.hip -- normalisation and error bars of the weighted first-passage histogram
// (Sec. 4.1), computed on the host from the histogram accumulators: a few numbers per slot, so
// no kernel.
//   fpt_density         P(deltaN) per bin, sum w / (n_traj width), and whole-run figures;
//   fpt_tail_at/_find   a tail set deltaN >= x*: its probability, error and ESS_T;
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

// ---------------------------------------------------------------------------
// Normalisation (Sec. 4.1): the density of deltaN per bin, whole-run figures and tail sets of a
// histogram read with fpt_histogram.  Host code: a few numbers per slot.
// ---------------------------------------------------------------------------
namespace {

// Checks shared by the normalisation calls: the histogram's arrays, the bin layout, a positive
// trajectory count and finite sums.
int check_hist(const fpt_hist *h, int32_t bins_kind, int32_t n_bins, double lo, double hi)
{
    if (!h || !h->count || !h->sum_w_bin || !h->sum_w2_bin) return report_error(FPT_EINVAL, "NULL histogram array");
    if (n_bins < 1 || n_bins > FPT_MAX_BINS) return report_error(FPT_EINVAL, "n_bins out of 1..FPT_MAX_BINS");
    if (bins_kind != FPT_BINS_LINEAR && bins_kind != FPT_BINS_LOG) return report_error(FPT_EINVAL, "bad bins_kind");
    if (!std::isfinite(lo) || !std::isfinite(hi) || !(hi > lo)) return report_error(FPT_EINVAL, "need finite lo < hi");
    if (bins_kind == FPT_BINS_LOG && !(lo > 0.0)) return report_error(FPT_EINVAL, "log bins need lo > 0");
    if (h->n_traj == 0) return report_error(FPT_EINVAL, "the histogram holds no trajectories");
    for (int j = 0; j < n_bins + 2; ++j)
        if (!std::isfinite(h->sum_w_bin[j]) || !std::isfinite(h->sum_w2_bin[j]))
            return report_error(FPT_EINVAL, "non-finite histogram sum");
    return FPT_OK;
}

// Edge e_j of the bins, j = 0 .. n_bins (the kernels bin with the same scale: t = (x - lo)
// n_bins/(hi - lo) or ln(x/lo) n_bins/ln(hi/lo)).
double bin_edge(int32_t bins_kind, int32_t n_bins, double lo, double hi, int j)
{
    if (j == n_bins) return hi;
    const double t = (double)j / (double)n_bins;
    return bins_kind == FPT_BINS_LINEAR ? lo + (hi - lo) * t : lo * std::pow(hi / lo, t);
}

void tail_from(const fpt_hist *h, int32_t bins_kind, int32_t n_bins, double lo, double hi, int slot, fpt_tail *out)
{
    double sw = 0.0, sw2 = 0.0;
    uint64_t c = 0;
    for (int j = n_bins + 1; j >= slot; --j) {
        sw += h->sum_w_bin[j];
        sw2 += h->sum_w2_bin[j];
        c += h->count[j];
    }
    const double n = (double)h->n_traj;
    out->slot = slot;
    out->x_star = bin_edge(bins_kind, n_bins, lo, hi, slot - 1);
    out->P = sw / n;
    out->P_err = std::sqrt(std::fmax(sw2 / n - out->P * out->P, 0.0) / n);
    out->ess = sw2 > 0.0 ? sw * sw / sw2 : 0.0;
    out->count = c;
    // the per-slot lognormal intervals of fpt_lognormal_bins, half-widths added in quadrature
    double q = 0.0;
    if (h->sum_lnw_bin && h->sum_lnw2_bin) {
        for (int j = slot; j <= n_bins + 1; ++j) {
            double p, lo_j, hi_j;
            if (fpt_lognormal_bins(1, h->n_traj, &h->count[j], &h->sum_lnw_bin[j], &h->sum_lnw2_bin[j], &p, &lo_j,
                                   &hi_j) != FPT_OK || !std::isfinite(hi_j - lo_j))
                continue;
            q += 0.25 * (hi_j - lo_j) * (hi_j - lo_j);
        }
    }
    out->P_err_lognormal = std::sqrt(q);
}

}  // namespace

extern "C" int fpt_density(const fpt_hist *h, int32_t bins_kind, int32_t n_bins, double lo, double hi,
                           double *density_out, double *edges_out, fpt_moments *m)
{
    const int rc = check_hist(h, bins_kind, n_bins, lo, hi);
    if (rc != FPT_OK) return rc;
    if (!density_out) return report_error(FPT_EINVAL, "NULL density_out");
    if (m && !(h->sum_w > 0.0 && std::isfinite(h->sum_w) && std::isfinite(h->sum_w2) && std::isfinite(h->sum_wN) &&
               std::isfinite(h->sum_wN2)))
        return report_error(FPT_EINVAL, "whole-run sums must be finite with sum_w > 0");
    const double n = (double)h->n_traj;
    double e0 = bin_edge(bins_kind, n_bins, lo, hi, 0);
    if (edges_out) edges_out[0] = e0;
    for (int j = 0; j < n_bins; ++j) {
        const double e1 = bin_edge(bins_kind, n_bins, lo, hi, j + 1);
        density_out[j] = h->sum_w_bin[j + 1] / (n * (e1 - e0));
        if (edges_out) edges_out[j + 1] = e1;
        e0 = e1;
    }
    if (m) {
        m->mean_w = h->sum_w / n;
        m->mean_N = h->sum_wN / h->sum_w;
        m->var_N = h->sum_wN2 / h->sum_w - m->mean_N * m->mean_N;
        m->ess = h->sum_w2 > 0.0 ? h->sum_w * h->sum_w / h->sum_w2 : 0.0;
        m->mass_under = h->sum_w_bin[0] / n;
        m->mass_over = h->sum_w_bin[n_bins + 1] / n;
    }
    return FPT_OK;
}

extern "C" int fpt_tail_at(const fpt_hist *h, int32_t bins_kind, int32_t n_bins, double lo, double hi, int32_t slot,
                           fpt_tail *out)
{
    const int rc = check_hist(h, bins_kind, n_bins, lo, hi);
    if (rc != FPT_OK) return rc;
    if (!out) return report_error(FPT_EINVAL, "NULL out");
    if (slot < 1 || slot > n_bins + 1) return report_error(FPT_EINVAL, "slot out of 1..n_bins + 1");
    tail_from(h, bins_kind, n_bins, lo, hi, slot, out);
    return FPT_OK;
}

extern "C" int fpt_tail_find(const fpt_hist *h, int32_t bins_kind, int32_t n_bins, double lo, double hi,
                             double p_target, fpt_tail *out)
{
    const int rc = check_hist(h, bins_kind, n_bins, lo, hi);
    if (rc != FPT_OK) return rc;
    if (!out) return report_error(FPT_EINVAL, "NULL out");
    if (!(p_target > 0.0) || !std::isfinite(p_target)) return report_error(FPT_EINVAL, "p_target must be > 0");
    // tail masses from the overflow slot down: the lowest slot whose mass is positive and at
    // most p_target (the masses do not decrease towards lower slots)
    const double n = (double)h->n_traj;
    double sw = 0.0;
    int best = -1;
    for (int j = n_bins + 1; j >= 1; --j) {
        sw += h->sum_w_bin[j];
        const double p = sw / n;
        if (p > p_target) break;
        if (p > 0.0) best = j;
    }
    if (best < 0) {
        *out = fpt_tail{-1, 0.0, 0.0, 0.0, 0.0, 0.0, 0};
        return FPT_OK;
    }
    tail_from(h, bins_kind, n_bins, lo, hi, best, out);
    return FPT_OK;
}
