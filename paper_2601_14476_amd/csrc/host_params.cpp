// host_params.cpp -- once-per-run parameters computed on the host: the I0
// schedule (Methods, experimental conditions) and the device-variability
// draw (Eq. 7).  Both are evaluated in double precision with a fixed
// operation order and rounded to single precision once.
#include <math.h>
#include <stdint.h>

#include "engine.hpp"

namespace psa {

// Philox4x32-10 on the host (Salmon et al., SC'11), for the variability draw.
void philox4x32_10_host(const uint32_t ctr[4], uint32_t k0, uint32_t k1, uint32_t out[4]) {
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    for (int round = 0; round < 10; ++round) {
        const uint64_t p0 = static_cast<uint64_t>(0xD2511F53u) * c0;
        const uint64_t p1 = static_cast<uint64_t>(0xCD9E8D57u) * c2;
        const uint32_t n0 = static_cast<uint32_t>(p1 >> 32) ^ c1 ^ k0;
        const uint32_t n2 = static_cast<uint32_t>(p0 >> 32) ^ c3 ^ k1;
        c1 = static_cast<uint32_t>(p1);
        c3 = static_cast<uint32_t>(p0);
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

// I0(0) = I0min, I0(t+1) = I0(t) / beta, beta = (I0min/I0max)^(1/(S-1)).
psa_status fill_schedule(int32_t steps, double i0_min, double i0_max, float *out) {
    if (steps < 1 || out == nullptr || !(i0_min > 0.0) || !(i0_max >= i0_min)) {
        set_error("schedule: need steps >= 1 and 0 < i0_min <= i0_max");
        return PSA_EINVAL;
    }
    if (steps == 1) {
        out[0] = static_cast<float>(i0_min);
        return PSA_OK;
    }
    const double beta = pow(i0_min / i0_max, 1.0 / static_cast<double>(steps - 1));
    double cur = i0_min;
    for (int32_t t = 0; t < steps; ++t) {
        out[t] = static_cast<float>(cur);
        cur = cur / beta;
    }
    return PSA_OK;
}

namespace {
// Standard normal from two words, Box-Muller cosine branch:
// u1 in (0,1], u2 in [0,1), z = sqrt(-2 ln u1) cos(2 pi u2).
double normal_from(uint32_t a, uint32_t b) {
    const double u1 = (static_cast<double>(a) + 1.0) / 4294967296.0;
    const double u2 = static_cast<double>(b) / 4294967296.0;
    return sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
}
}  // namespace

psa_status draw_variability(int32_t n, uint64_t seed, double sigma_lambda, double sigma_delta,
                            double sigma_nu, double p_mean, float *lambda, float *delta,
                            uint32_t *thr24) {
    if (n < 1 || !lambda || !delta || !thr24) {
        set_error("variability: need n >= 1 and non-null outputs");
        return PSA_EINVAL;
    }
    if (!(sigma_lambda >= 0.0) || !(sigma_delta >= 0.0) || !(sigma_nu >= 0.0) ||
        !(p_mean >= 0.0 && p_mean <= 1.0)) {
        set_error("variability: sigmas must be >= 0 and p_mean in [0, 1]");
        return PSA_EINVAL;
    }
    const uint32_t k0 = static_cast<uint32_t>(seed);
    const uint32_t k1 = static_cast<uint32_t>(seed >> 32);
    for (int32_t i = 0; i < n; ++i) {
        const uint32_t ca[4] = {0u, static_cast<uint32_t>(i), 0u, kTagVarHost};
        const uint32_t cb[4] = {0u, static_cast<uint32_t>(i), 1u, kTagVarHost};
        uint32_t a[4], b[4];
        philox4x32_10_host(ca, k0, k1, a);
        philox4x32_10_host(cb, k0, k1, b);
        const double z_lambda = normal_from(a[0], a[1]);
        const double z_delta = normal_from(a[2], a[3]);
        const double z_nu = normal_from(b[0], b[1]);
        lambda[i] = static_cast<float>(1.0 + sigma_lambda * z_lambda);
        delta[i] = static_cast<float>(sigma_delta * z_delta);
        double p = p_mean + sigma_nu * z_nu;
        p = p < 0.0 ? 0.0 : (p > 1.0 ? 1.0 : p);
        thr24[i] = static_cast<uint32_t>(floor(p * 16777216.0));
    }
    return PSA_OK;
}

psa_status draw_periods(int32_t n, uint64_t seed, double sigma_nu, int32_t t_res,
                        uint32_t *period) {
    if (n < 1 || !period || t_res < 1 || !(sigma_nu >= 0.0)) {
        set_error("periods: need n >= 1, t_res >= 1, sigma_nu >= 0 and an output");
        return PSA_EINVAL;
    }
    const uint32_t k0 = static_cast<uint32_t>(seed);
    const uint32_t k1 = static_cast<uint32_t>(seed >> 32);
    for (int32_t i = 0; i < n; ++i) {
        const uint32_t cb[4] = {0u, static_cast<uint32_t>(i), 1u, kTagVarHost};
        uint32_t b[4];
        philox4x32_10_host(cb, k0, k1, b);
        const double nu = sigma_nu * normal_from(b[0], b[1]);
        const double p = rint(static_cast<double>(t_res) * (1.0 + nu));
        period[i] = p < 1.0 ? 1u : static_cast<uint32_t>(p);
    }
    return PSA_OK;
}

}  // namespace psa
