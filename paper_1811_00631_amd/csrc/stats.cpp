// stats.cpp -- significance of IG^k_max on the host, in binary64.
//
// Section "Theory", the paragraphs after equation IGmax: for an irrelevant variable and one
// k-tuple, IG (in nats, times N) is chi-square distributed for large samples; IG^k_max, the
// largest of many such values, follows an extreme value distribution whose one free parameter
// is the number of independent tests, fitted to the irrelevant part of the data; this turns
// IG^k_max into a p-value and gives IG_lim for a significance level, and the p-values of many
// variables are adjusted by Holm (FWER) or Benjamini-Hochberg / Benjamini-Hochberg-Yekutieli
// (FDR) (section "Canonical package usage": ComputePValue, then p.adjust).
//
// Readings (the fit itself is specified in a companion paper that is not available):
//   * 2 IG of one tuple ~ chi-square with df = (c-1) c^(k-1), c = divisions + 1 classes per
//     variable and a binary decision (the contingency table of y against the tuple's c^k cells
//     less the constraints of its margins).
//   * IG^k_max of an irrelevant variable is the maximum of n_eff independent such values:
//     Pr(IG_max <= x) = F(2x)^n_eff with F the chi-square CDF.  Its density is
//     n_eff F^(n_eff-1) f, so the maximum likelihood estimate over m irrelevant variables has a
//     closed form: n_eff = -m / sum ln F(2 x_v).  Values x_v <= 0 have probability 0 under the
//     model and are left out of the fit (their p-value is 1).
//   * p-value = 1 - F(2x)^n_eff, evaluated as -expm1(n_eff ln F(2x)) with ln F from whichever
//     tail is accurate, so p-values far below 1e-16 keep their relative precision.
//
// F(2x) for df degrees of freedom is the regularised lower incomplete gamma function
// P(df/2, x).  It is evaluated by the power series of P for x < a + 1 and by the continued
// fraction of Q = 1 - P (modified Lentz evaluation) otherwise, the standard pair of methods
// (Press, Teukolsky, Vetterling and Flannery, "Numerical Recipes", section on the incomplete
// gamma function); the code here is written from those formulas.
#include "mdfs.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <numeric>
#include <string>
#include <vector>

namespace mdfs {
void set_error(const char *msg);   // api.hip: thread-local message for mdfs_last_error
}

namespace {

// ln P(a, x) and ln Q(a, x) for a > 0, x > 0.
void log_pq(double a, double x, double &lnP, double &lnQ)
{
    const double lnpre = a * std::log(x) - x - std::lgamma(a);   // ln(x^a e^-x / Gamma(a))
    if (x < a + 1.0) {
        // P = x^a e^-x / Gamma(a + 1) * sum_n x^n / ((a+1)...(a+n))
        double term = 1.0 / a, sum = term;
        for (int n = 1; n < 100000; ++n) {
            term *= x / (a + n);
            sum += term;
            if (std::fabs(term) < std::fabs(sum) * 1e-17) break;
        }
        lnP = lnpre + std::log(sum);
        lnQ = std::log1p(-std::exp(lnP));
    } else {
        // Q = x^a e^-x / Gamma(a) * 1 / (x + 1 - a - 1 (1 - a) / (x + 3 - a - 2 (2 - a) / ...))
        const double tiny = 1e-300;
        double b = x + 1.0 - a, c = 1.0 / tiny, d = 1.0 / b, h = d;
        for (int i = 1; i < 100000; ++i) {
            const double an = -i * (i - a);
            b += 2.0;
            d = an * d + b;
            if (std::fabs(d) < tiny) d = tiny;
            c = b + an / c;
            if (std::fabs(c) < tiny) c = tiny;
            d = 1.0 / d;
            const double del = d * c;
            h *= del;
            if (std::fabs(del - 1.0) < 1e-16) break;
        }
        lnQ = lnpre + std::log(h);
        lnP = std::log1p(-std::exp(lnQ));
    }
}

// ln F(2x) for df degrees of freedom, F the chi-square CDF; -inf for x <= 0.
double ln_cdf2(double x, int df)
{
    if (!(x > 0.0)) return -INFINITY;
    if (std::isinf(x)) return 0.0;
    double lnP, lnQ;
    log_pq(0.5 * df, x, lnP, lnQ);
    return lnP;
}

// 1 - exp(n lnF), accurate when n lnF is tiny
double pvalue_of(double lnF, double n_eff)
{
    if (lnF == -INFINITY) return 1.0;
    return -std::expm1(n_eff * lnF);
}

}  // namespace

extern "C" {

int mdfs_chi2_df(int k, int divisions)
{
    if (k < 1 || k > 5) {
        mdfs::set_error("k must be in [1, 5]");
        return MDFS_E_K;
    }
    if (divisions < 1 || divisions > 15) {
        mdfs::set_error("divisions must be in [1, 15]");
        return MDFS_E_DIV;
    }
    const int c = divisions + 1;
    int df = c - 1;
    for (int i = 1; i < k; ++i) df *= c;
    mdfs::set_error("");
    return df;
}

int mdfs_pvalues(const double *ig, int64_t n, int k, int divisions, const uint8_t *fit_mask, double n_eff_fixed,
                 double *p_out, double *n_eff_out)
{
    const int df = mdfs_chi2_df(k, divisions);
    if (df < 0) return df;
    if (!ig || !p_out || n < 1) {
        mdfs::set_error("ig and p_out must be non-null and n >= 1");
        return MDFS_E_ARG;
    }
    if (std::isnan(n_eff_fixed)) {
        mdfs::set_error("n_eff_fixed is NaN");
        return MDFS_E_ARG;
    }
    std::vector<double> lnF((size_t)n);
    for (int64_t v = 0; v < n; ++v) {
        if (std::isnan(ig[v])) {
            mdfs::set_error("ig holds a NaN");
            return MDFS_E_ARG;
        }
        lnF[(size_t)v] = ln_cdf2(ig[v], df);
    }
    double n_eff = n_eff_fixed;
    if (!(n_eff_fixed > 0.0)) {
        double s = 0.0;
        int64_t m = 0;
        for (int64_t v = 0; v < n; ++v) {
            if (fit_mask && !fit_mask[v]) continue;
            if (lnF[(size_t)v] == -INFINITY) continue;   // IG <= 0: outside the model's support
            s += lnF[(size_t)v];
            ++m;
        }
        if (m == 0 || !(s < 0.0)) {
            mdfs::set_error("no variable with 0 < IG < inf selected for the fit");
            return MDFS_E_ARG;
        }
        n_eff = -(double)m / s;
    }
    for (int64_t v = 0; v < n; ++v) p_out[v] = pvalue_of(lnF[(size_t)v], n_eff);
    if (n_eff_out) *n_eff_out = n_eff;
    mdfs::set_error("");
    return MDFS_OK;
}

int mdfs_ig_lim(int k, int divisions, double n_eff, double alpha, double *ig_lim)
{
    const int df = mdfs_chi2_df(k, divisions);
    if (df < 0) return df;
    if (!ig_lim || !(n_eff > 0.0) || std::isinf(n_eff) || !(alpha > 0.0 && alpha < 1.0)) {
        mdfs::set_error("need ig_lim non-null, 0 < n_eff < inf and 0 < alpha < 1");
        return MDFS_E_ARG;
    }
    // the x with n_eff ln F(2x) = ln(1 - alpha): ln F is increasing, bracket and bisect
    const double target = std::log1p(-alpha) / n_eff;
    double lo = 0.0, hi = 1.0;
    while (ln_cdf2(hi, df) < target) {
        lo = hi;
        hi *= 2.0;
        if (hi > 1e300) {
            mdfs::set_error("IG_lim out of range");
            return MDFS_E_ARG;
        }
    }
    for (int it = 0; it < 200 && hi - lo > 1e-15 * hi; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (ln_cdf2(mid, df) < target) lo = mid;
        else hi = mid;
    }
    *ig_lim = 0.5 * (lo + hi);
    mdfs::set_error("");
    return MDFS_OK;
}

int mdfs_p_adjust(const double *p, int64_t n, int method, double *out)
{
    if (!p || !out || n < 1) {
        mdfs::set_error("p and out must be non-null and n >= 1");
        return MDFS_E_ARG;
    }
    if (method < MDFS_ADJ_NONE || method > MDFS_ADJ_BY) {
        mdfs::set_error("unknown adjustment method");
        return MDFS_E_ARG;
    }
    for (int64_t v = 0; v < n; ++v)
        if (std::isnan(p[v]) || p[v] < 0.0 || p[v] > 1.0) {
            mdfs::set_error("p-values must lie in [0, 1]");
            return MDFS_E_ARG;
        }
    std::vector<int64_t> ord((size_t)n);
    std::iota(ord.begin(), ord.end(), (int64_t)0);
    // ascending p, ties by index (the adjusted values do not depend on the tie order)
    std::stable_sort(ord.begin(), ord.end(), [&](int64_t x, int64_t y) { return p[x] < p[y]; });
    const double nn = (double)n;
    if (method == MDFS_ADJ_NONE) {
        for (int64_t v = 0; v < n; ++v) out[v] = p[v];
    } else if (method == MDFS_ADJ_HOLM) {
        // (n - i) p_(i) for 0-based rank i, running maximum from the smallest p, capped at 1
        double run = 0.0;
        for (int64_t i = 0; i < n; ++i) {
            run = std::max(run, std::min(1.0, (nn - (double)i) * p[ord[(size_t)i]]));
            out[ord[(size_t)i]] = run;
        }
    } else {
        // n / (i + 1) p_(i) (times sum_{j<=n} 1/j for BY), running minimum from the largest p
        double cn = 1.0;
        if (method == MDFS_ADJ_BY) {
            cn = 0.0;
            for (int64_t j = n; j >= 1; --j) cn += 1.0 / (double)j;
        }
        double run = 1.0;
        for (int64_t i = n - 1; i >= 0; --i) {
            run = std::min(run, std::min(1.0, cn * nn / (double)(i + 1) * p[ord[(size_t)i]]));
            out[ord[(size_t)i]] = run;
        }
    }
    mdfs::set_error("");
    return MDFS_OK;
}

}  // extern "C"
