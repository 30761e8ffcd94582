"""Ensemble observables on the device: the ageing overlap of Sec. VIII B,
Eq. (68), C(t_w, dt_w) = <sum_r phi(t_w) phi(t_w + dt_w)> / <sum_r phi(t_w)^2>,
phi = rho_A - rho_B, with the brackets over realizations.  Each lattice keeps
phi(t_w) on the device (lb_set_overlap_reference) and its observables carry
the two site sums in FP64; the ensemble ratio is the sum over lattices of
the first over the sum of the second.  Checked against the oracle's fields
for a small ensemble of uneven lattices, batched against alone bit for bit."""
import numpy as np
import pytest
import torch  # noqa: F401  (first import can be slow; keep it out of test timeouts)

import oracle
from paper_0906_3611_amd import analysis, inputs

pytestmark = pytest.mark.gpu

C1 = dict(tau=(1.0, 1.0), rho0=0.83, G_a=(-9.0, -9.0), G_r=(8.1, 8.1), G_AB=0.405)
SHAPES = ((48, 40), (64, 64), (40, 56), (72, 33))
T_W, DT = 300, 200


def _lb():
    from paper_0906_3611_amd import lb
    return lb


def _fields(k, nx, ny):
    """Disc emulsions (the C2 recipe at phi = 0.6, seed 70 + k)."""
    return inputs.disc_fields(nx, ny, 70 + k, 0.6)


def _oracle_sums():
    out = []
    for k, (nx, ny) in enumerate(SHAPES):
        p = oracle.Params(nx=nx, ny=ny, tau=C1["tau"], rho0=C1["rho0"], Ga=C1["G_a"], Gr=C1["G_r"],
                          Gab=C1["G_AB"])
        f, _ = oracle.run(p, oracle.init_equilibrium(p, *_fields(k, nx, ny)), T_W)
        phi_w = analysis.order_parameter(oracle.density(p, f))
        f, _ = oracle.run(p, f, DT)
        phi_t = analysis.order_parameter(oracle.density(p, f))
        out.append((phi_w, phi_t))
    return out


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32dev", 1e-5), ("fp32mom", 1e-5)])
def test_overlap_sums_against_the_oracle(precision, tol):
    lb = _lb()
    b = lb.Batch([dict(C1, nx=nx, ny=ny, precision=precision) for nx, ny in SHAPES])
    for k, (nx, ny) in enumerate(SHAPES):
        b.init(k, *_fields(k, nx, ny))
    assert all(o["ref_step"] == -1 and o["phi_ref_sq"] == 0.0 for o in b.observables())
    b.step(T_W)
    b.set_overlap_reference()
    at_w = b.observables()
    for o in at_w:   # at t_w the overlap is the norm itself, bit for bit
        assert o["ref_step"] == T_W and o["phi_overlap"] == o["phi_ref_sq"] > 0
    b.step(DT)
    obs = b.observables()
    ref = _oracle_sums()
    for o, (phi_w, phi_t) in zip(obs, ref):
        assert o["ref_step"] == T_W and o["step"] == T_W + DT
        assert o["phi_ref_sq"] == pytest.approx(np.sum(phi_w * phi_w), rel=tol)
        assert o["phi_overlap"] == pytest.approx(np.sum(phi_w * phi_t), rel=tol)
    c_dev = sum(o["phi_overlap"] for o in obs) / sum(o["phi_ref_sq"] for o in obs)
    c_ref = analysis.overlap(np.concatenate([w.ravel() for w, _ in ref]),
                             np.concatenate([t.ravel() for _, t in ref]))
    assert 0.0 < c_ref < 1.0   # the coarsening pattern decorrelates
    assert c_dev == pytest.approx(c_ref, rel=tol)
    b.close()


def test_overlap_alone_equals_batched_bitwise():
    lb = _lb()
    b = lb.Batch([dict(C1, nx=nx, ny=ny, precision="fp32dev") for nx, ny in SHAPES])
    for k, (nx, ny) in enumerate(SHAPES):
        b.init(k, *_fields(k, nx, ny))
    b.step(T_W)
    b.set_overlap_reference()
    b.step(DT)
    batched = b.observables()
    b.close()
    for k, (nx, ny) in enumerate(SHAPES):
        lat = lb.Lattice(nx, ny, precision="fp32dev", **C1)
        lat.init(*_fields(k, nx, ny))
        lat.step(T_W)
        lat.set_overlap_reference()
        lat.step(DT)
        o = lat.observables()
        for key in ("phi_overlap", "phi_ref_sq", "ref_step", "mass"):
            assert np.array_equal(o[key], batched[k][key]), (k, key)
        # a new initial state drops the reference
        lat.init(*_fields(k, nx, ny))
        o = lat.observables()
        assert o["ref_step"] == -1 and o["phi_overlap"] == 0.0
        lat.close()
