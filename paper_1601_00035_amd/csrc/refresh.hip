// Cadence of the velocity refresh (Sec. 4.4) from the truncation error of the masked integrating
// factor (Appendix D), evaluated on the host.
//
// For a uniform field on a half-space whose mask keeps the points k >= 1 along one axis, the masked
// integrating factor loses at the point k the mass of the 1D kernel w_a[n] = e^{-2a} I_n(2a) at
// distances n >= k:  d_a(k) = sum_{n >= k} w_a[n].  The integrating factors of q steps compose to
// E(q beta), beta = dt / (dx^2 Re), and the solution domain starts n_buf points inside the box
// (k = n_buf + 1), so the error there after q steps is estimated by umax d_{q beta}(n_buf + 1).
#include <cmath>

#include "kernels.h"

namespace nslgf {

// w_a[n] = e^{-2a} I_n(2a) = sum_j a^{2j+n} e^{-2a} / (j! (j+n)!), all terms positive.  The largest
// term (where a^2 = j (j + n)) is evaluated in log space and the others by the ratio of consecutive
// terms, a^2 / ((j + 1)(j + n + 1)), outwards from it, so no intermediate overflows for any a.
static double scaled_bessel_i(double a, int n) {
    const double la = std::log(a);
    const double jr = 0.5 * (-(double)n + std::sqrt((double)n * n + 4.0 * a * a));
    const double jp = std::floor(jr);
    const double peak = std::exp((2.0 * jp + n) * la - std::lgamma(jp + 1.0) - std::lgamma(jp + n + 1.0) - 2.0 * a);
    double sum = peak;
    double t = peak;
    for (double j = jp; t > 1e-18 * sum; j += 1.0) {  // upwards: t_{j+1} = t_j a^2 / ((j+1)(j+n+1))
        t *= a * a / ((j + 1.0) * (j + n + 1.0));
        sum += t;
    }
    t = peak;
    for (double j = jp; j > 0.0 && t > 1e-18 * sum; j -= 1.0) {  // downwards: t_{j-1} = t_j j (j+n) / a^2
        t *= j * (j + n) / (a * a);
        sum += t;
    }
    return sum;
}

double if_trunc_error_host(double alpha, int k) {
    if (alpha == 0.0) return 0.0;
    // w_a[n] decreases in n >= 0: add terms until they no longer change the sum
    double sum = 0.0;
    for (long long n = k; n < (long long)k + 10000000; ++n) {
        const double t = scaled_bessel_i(alpha, (int)n);
        sum += t;
        if (t <= 1e-18 * sum) break;
    }
    return sum;
}

int refresh_interval_host(double beta, int n_buf, double umax, double eps, int q_cap) {
    if (umax == 0.0 || beta == 0.0) return q_cap;
    // d_a(k) < d_a(1) = (1 - w_a[0]) / 2 < 1/2 for every a: nothing to search when eps allows that
    if (eps >= 0.5 * umax) return q_cap;
    auto ok = [&](long long q) { return umax * if_trunc_error_host((double)q * beta, n_buf + 1) <= eps; };
    if (!ok(1)) return 0;
    // the estimate grows with q: double to bracket the first failing q, then bisect
    long long lo = 1, hi = 2;
    while (hi <= q_cap && ok(hi)) {
        lo = hi;
        hi *= 2;
    }
    if (hi > q_cap) {
        if (ok(q_cap)) return q_cap;
        hi = q_cap;
    }
    while (hi - lo > 1) {  // ok(lo), !ok(hi)
        const long long mid = lo + (hi - lo) / 2;
        if (ok(mid))
            lo = mid;
        else
            hi = mid;
    }
    return (int)lo;
}

}  // namespace nslgf
