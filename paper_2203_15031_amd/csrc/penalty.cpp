// penalty.cpp -- the penalty levels of Section 2.2 (host code).
//
//   lambda_univ = sqrt(2 log(p-1) / n)       (universal level, as the worked
//                                             example of Section 2.2 evaluates it)
//   lambda_ub   = sqrt(4 log p / n)          (union bound over p scaled lassos)
//   lambda_pb   = sqrt(2) L_n(k/p), L_n(t) = n^-1/2 Phi^-1(1 - t), with k the
//                 root in (0, p/2) of k = L_1^4(k/p) + 2 L_1^2(k/p), found by
//                 the bisection method the paper names.
//
// Phi^-1 is Wichura's algorithm AS 241 (PPND16, Applied Statistics 37, 1988),
// accurate to about 1e-16 relative.
#include <math.h>

#include "spmesl.h"

namespace {

double poly(const double *c, int deg, double x)
{
    double v = c[deg];
    for (int i = deg - 1; i >= 0; --i) v = v * x + c[i];
    return v;
}

// AS 241 PPND16: Phi^-1(p) for 0 < p < 1.
double norm_quantile(double p)
{
    static const double a[8] = {3.3871328727963666080e0, 1.3314166789178437745e+2,
                                1.9715909503065514427e+3, 1.3731693765509461125e+4,
                                4.5921953931549871457e+4, 6.7265770927008700853e+4,
                                3.3430575583588128105e+4, 2.5090809287301226727e+3};
    static const double b[8] = {1.0, 4.2313330701600911252e+1, 6.8718700749205790830e+2,
                                5.3941960214247511077e+3, 2.1213794301586595867e+4,
                                3.9307895800092710610e+4, 2.8729085735721942674e+4,
                                5.2264952788528545610e+3};
    static const double c[8] = {1.42343711074968357734e0, 4.63033784615654529590e0,
                                5.76949722146069140550e0, 3.64784832476320460504e0,
                                1.27045825245236838258e0, 2.41780725177450611770e-1,
                                2.27238449892691845833e-2, 7.74545014278341407640e-4};
    static const double d[8] = {1.0, 2.05319162663775882187e0, 1.67638483018380384940e0,
                                6.89767334985100004550e-1, 1.48103976427480074590e-1,
                                1.51986665636164571966e-2, 5.47593808499534494600e-4,
                                1.05075007164441684324e-9};
    static const double e[8] = {6.65790464350110377720e0, 5.46378491116411436990e0,
                                1.78482653991729133580e0, 2.96560571828504891230e-1,
                                2.65321895265761230930e-2, 1.24266094738807843860e-3,
                                2.71155556874348757815e-5, 2.01033439929228813265e-7};
    static const double f[8] = {1.0, 5.99832206555887937690e-1, 1.36929880922735805310e-1,
                                1.48753612908506148525e-2, 7.86869131145613259100e-4,
                                1.84631831751005468180e-5, 1.42151175831644588870e-7,
                                2.04426310338993978564e-15};
    double q = p - 0.5;
    if (fabs(q) <= 0.425) {
        double r = 0.180625 - q * q;
        return q * poly(a, 7, r) / poly(b, 7, r);
    }
    double r = q < 0.0 ? p : 1.0 - p;
    r = sqrt(-log(r));
    double v;
    if (r <= 5.0) {
        r -= 1.6;
        v = poly(c, 7, r) / poly(d, 7, r);
    } else {
        r -= 5.0;
        v = poly(e, 7, r) / poly(f, 7, r);
    }
    return q < 0.0 ? -v : v;
}

double L_n(double n, double t) { return norm_quantile(1.0 - t) / sqrt(n); }

} // namespace

extern "C" double spmesl_lambda_univ(double n, double p)
{
    if (!(n > 0.0) || !(p > 2.0)) return NAN;
    return sqrt(2.0 * log(p - 1.0) / n);
}

extern "C" double spmesl_lambda_ub(double n, double p)
{
    if (!(n > 0.0) || !(p > 1.0)) return NAN;
    return sqrt(4.0 * log(p) / n);
}

extern "C" int spmesl_lambda_pb(double n, double p, double *lambda_out, double *k_out)
{
    if (!(n > 0.0) || !(p >= 2.0) || !lambda_out) return SPMESL_EINVAL;
    // h(k) = k - L_1^4(k/p) - 2 L_1^2(k/p) is negative near 0 and equals p/2 at
    // k = p/2; bisect on the sign change.
    double lo = 0.0, hi = 0.5 * p;
    for (int it = 0; it < 300 && hi - lo > 1e-15 * hi; ++it) {
        double mid = 0.5 * (lo + hi);
        if (mid <= 0.0) break;
        double L = L_n(1.0, mid / p);
        double h = mid - (L * L * L * L + 2.0 * L * L);
        if (h < 0.0) lo = mid;
        else hi = mid;
    }
    double k = 0.5 * (lo + hi);
    *lambda_out = sqrt(2.0) * L_n(n, k / p);
    if (k_out) *k_out = k;
    return SPMESL_OK;
}
