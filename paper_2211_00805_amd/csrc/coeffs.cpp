// Chebyshev coefficients of the heat kernel (Sec. "Chebyshev Polynomials").
//
// exp(-t(y+1)) = sum' b_k T_k(y) on [-1, 1] with b_k = 2 (-1)^k e^{-t} I_k(t):
// the generating function exp(z cos th) = I_0(z) + 2 sum_k I_k(z) cos(k th)
// taken at z = -t.  e^{-t} I_k(t) is evaluated by Miller's backward
// recurrence I_{k-1} = (2k/t) I_k + I_{k+1}, started far above the largest
// order needed and normalised with the identity e^t = I_0 + 2 sum_{k>=1} I_k,
// which makes the exponentially scaled values come out directly.
#include <cmath>
#include <vector>

#include "internal.h"

namespace gs {

void bessel_ive_table(double t, int kmax, std::vector<double>& out) {
    out.assign(kmax + 1, 0.0);
    if (t == 0.0) {
        out[0] = 1.0;
        return;
    }
    const int N = std::max(kmax + 1, (int)(t + 12.0 * std::sqrt(t + 1.0))) + 40 +
                  (int)std::sqrt(40.0 * (kmax + 1));
    std::vector<double> f(N + 2, 0.0);
    f[N + 1] = 0.0;
    f[N] = 1e-30;
    for (int k = N; k >= 1; --k) {
        f[k - 1] = (2.0 * k / t) * f[k] + f[k + 1];
        if (std::fabs(f[k - 1]) > 1e250) {  // rescale what has been computed so far
            for (int j = k - 1; j <= N; ++j) f[j] *= 1e-250;
        }
    }
    double norm = f[0];
    for (int k = 1; k <= N; ++k) norm += 2.0 * f[k];
    for (int k = 0; k <= kmax; ++k) out[k] = f[k] / norm;
}

void cheby_coeffs(double t, int K, double* b, double* db) {
    std::vector<double> ive;
    bessel_ive_table(t, K + 1, ive);
    for (int k = 0; k <= K; ++k) {
        const double sgn = (k % 2) ? -1.0 : 1.0;
        b[k] = 2.0 * sgn * ive[k];
        if (db) {
            const double im1 = ive[k == 0 ? 1 : k - 1];
            db[k] = 2.0 * sgn * (0.5 * (im1 + ive[k + 1]) - ive[k]);
        }
    }
}

double cheby_tail(double t, int K) {
    const int extra = 400;
    std::vector<double> ive;
    bessel_ive_table(t, K + extra, ive);
    double s = 0.0;
    for (int k = K + extra; k > K; --k) s += 2.0 * ive[k];
    return s;
}

}  // namespace gs
