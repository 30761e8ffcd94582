"""The FP32 expm1 used for psi on the device (range reduction plus a Taylor
polynomial, `expm1_rr` in the device helpers) restated step by step in
float32 on the host, against FP64 expm1: at most 1.5 ulp over the densities
a lattice can hold.  This pins the constants and the error bound of the
method; the GPU parity tests cover the compiled code."""
import numpy as np

F = np.float32


def _fma(a, b, c):
    # products of two float32 are exact in float64: one rounding to float32
    return F(np.float64(a) * np.float64(b) + np.float64(c))


def _expm1_steps(x):
    x = F(x)
    k = F(np.rint(F(x * F(1.44269504))))
    t = _fma(-k, F(0.693145751953125), x)
    t = _fma(-k, F(1.42860677e-06), t)
    b = F(1 / 5040)
    for c in (1 / 720, 1 / 120, 1 / 24, 1 / 6, 0.5):
        b = _fma(b, t, F(c))
    p = _fma(F(t * t), b, t)
    s = F(np.ldexp(F(1), int(k)))
    return _fma(s, p, F(s - F(1)))


def test_ln2_split_is_exact_for_the_reduction():
    hi = F(0.693145751953125)
    # 16 significant bits: k * hi is exact for |k| < 2^8
    assert float(hi) * 256 == float(F(float(hi) * 256))
    assert abs(float(hi) + float(F(1.42860677e-06)) - np.log(2)) < 1e-12


def test_within_1p5_ulp_of_fp64_expm1():
    rng = np.random.default_rng(7)
    xs = np.concatenate([np.linspace(-20, 5, 20001), rng.uniform(-3, 3, 20000),
                         np.linspace(-1e-3, 1e-3, 2001), -np.logspace(-8, 0, 401),
                         np.logspace(-8, 0, 401), [0.0]]).astype(np.float32)
    worst = 0.0
    for x in xs:
        ref = np.expm1(np.float64(x))
        got = np.float64(_expm1_steps(x))
        if ref == 0.0:
            assert got == 0.0
            continue
        worst = max(worst, abs(got - ref) / float(np.spacing(F(ref))))
    assert worst <= 1.5, worst
