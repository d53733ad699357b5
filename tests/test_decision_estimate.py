"""The p-bit decision's estimate-first shortcut (CPU check of its error bound).

The kernels decide +1 iff tanh_f32(x) > r, where tanh_f32 is the library's
fixed single-precision recipe (degree-7 polynomial for 2^f, ldexp, a
correctly rounded 2 / (e + 1)).  They first form a cheap estimate of the same
value from the hardware 2^v and reciprocal (each within about one ulp) and
decide from it alone when it lies more than 2^-16 from r; the exact recipe
decides the rest.  That is exact only if the estimate is always within 2^-16
of the recipe.  This test evaluates the recipe in float32 (fused multiply-adds
emulated in float64, which is exact for these products), perturbs the
estimate's 2^v and reciprocal by up to 4 ulp each (twice the documented
hardware error), and checks the distance over a dense sweep of x, with a
factor of 8 to spare against the margin.
"""
import numpy as np

f32 = np.float32
MARGIN = 2.0 ** -16

# Taylor coefficients of e^(f ln 2), rounded to float (the recipe's table)
COEF = [float.fromhex(h) for h in ("0x1.ffcbfcp-17", "0x1.430912p-13", "0x1.5d87fep-10",
                                   "0x1.3b2ab6p-7", "0x1.c6b08ep-5", "0x1.ebfbe0p-3",
                                   "0x1.62e430p-1")]
LOG2E_2 = f32(float.fromhex("0x1.715476p+1"))


def tanh_recipe(x):
    """The recipe, operation by operation, in float32."""
    a = np.minimum(np.abs(x), f32(9.0)).astype(f32)
    v = (a * LOG2E_2).astype(f32)
    nf = np.rint(v).astype(f32)
    f = (v - nf).astype(f32)
    p = np.full_like(f, f32(COEF[0]))
    for c in COEF[1:] + [1.0]:
        p = (p.astype(np.float64) * f.astype(np.float64) + c).astype(f32)   # fmaf
    e = np.ldexp(p, nf.astype(np.int32)).astype(f32)
    q = (f32(2.0) / (e + f32(1.0)).astype(f32)).astype(f32)
    y = (f32(1.0) - q).astype(f32)
    y = np.where(a >= f32(9.0), f32(1.0), y)
    return np.copysign(y, x).astype(f32)


def estimate(x, exp_ulps, rcp_ulps):
    """The estimate with its 2^v and reciprocal off by the given ulps."""
    a = np.minimum(np.abs(x), f32(9.0)).astype(f32)
    v = (a * LOG2E_2).astype(f32)
    e = np.exp2(v.astype(np.float64)).astype(f32)
    e = (e.astype(np.float64) * (1.0 + exp_ulps * 2.0 ** -23)).astype(f32)
    d = (e + f32(1.0)).astype(f32)
    rc = (1.0 / d.astype(np.float64)).astype(f32)
    rc = (rc.astype(np.float64) * (1.0 + rcp_ulps * 2.0 ** -23)).astype(f32)
    y = (-2.0 * rc.astype(np.float64) + 1.0).astype(f32)                     # fmaf
    return np.copysign(y, x).astype(f32)


def test_estimate_within_margin():
    rng = np.random.default_rng(3)
    x = np.concatenate([
        np.linspace(-9.5, 9.5, 200001),
        rng.normal(0.0, 0.3, 100000),
        rng.uniform(-1e-3, 1e-3, 20000),
        np.array([0.0, -0.0, 9.0, -9.0, 8.999999, 1e-30, -1e-30]),
    ]).astype(f32)
    y = tanh_recipe(x).astype(np.float64)
    worst = 0.0
    for eu in (-4, 0, 4):
        for ru in (-4, 0, 4):
            worst = max(worst, float(np.max(np.abs(estimate(x, eu, ru).astype(np.float64) - y))))
    assert worst < MARGIN / 8, worst


def test_recipe_is_tanh():
    """The recipe itself is tanh to within a few float32 ulps (so the
    estimate is an estimate of tanh, not of something else)."""
    x = np.linspace(-12.0, 12.0, 100001).astype(f32)
    err = np.abs(tanh_recipe(x).astype(np.float64) - np.tanh(x.astype(np.float64)))
    assert float(err.max()) < 4 * 2.0 ** -24, float(err.max())
