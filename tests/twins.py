"""Error envelopes from the oracle (test helpers; they call only oracle/).

A twin is the FP64 oracle run again with a perturbation of rounding size.
Where the dynamics amplify rounding (the demixing pattern of C1, the
coarsening emulsion of C2) the distance between a twin and the plain oracle
run measures how far two correct evaluations of the same model may drift
apart, so an FP32 result is judged against it rather than against a fixed
number.
"""
import numpy as np

import oracle

# D2Q9 weights (Table I) in the oracle's direction order
W9 = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)


def deviation_refs(f0: np.ndarray) -> np.ndarray:
    """Per-species reference densities of the FP32 deviation storage: the
    lattice mean of the initial densities, rounded to FP32."""
    rho = f0.sum(axis=1)
    return np.array([float(np.float32(rho[s].mean())) for s in range(2)])


def round_to_storage(f: np.ndarray, rref: np.ndarray) -> np.ndarray:
    """The populations as the FP32 deviation storage holds them:
    w_i rho_ref_s + fl32(f_is - w_i rho_ref_s)."""
    base = W9[None, :, None, None] * rref[:, None, None, None]
    return base + (f - base).astype(np.float32).astype(np.float64)


def storage_rounding_twin(p, f0: np.ndarray, steps: int, checkpoints=None):
    """The oracle with its state rounded to the FP32 deviation storage after
    the initial state and after every step: the rounding the storage itself
    adds each step, without FP32 arithmetic.  Returns the state after
    `steps` steps, or a list of states at the given checkpoints."""
    rref = deviation_refs(f0)
    f = round_to_storage(f0, rref)
    out, want = [], set(checkpoints or [])
    for t in range(1, steps + 1):
        f = round_to_storage(oracle.step(p, f), rref)
        if t in want:
            out.append(f.copy())
    return out if checkpoints else f


def noise_twin_start(f0: np.ndarray, seed: int, rel: float = 2.0 ** -24) -> np.ndarray:
    """f0 with every population of both species multiplied by an independent
    1 + e, e uniform in [-rel, rel) (FP32 unit roundoff by default)."""
    rng = np.random.default_rng(seed)
    return f0 * (1.0 + rel * (2.0 * rng.random(f0.shape) - 1.0))


def arithmetic_rounding_twin(p, f0: np.ndarray, steps: int, seed: int, checkpoints=None,
                             rel: float = 2.0 ** -24):
    """The oracle with every population multiplied by an independent
    1 + e, e uniform in [-rel, rel), after every step: rounding at the scale
    of the populations themselves, as FP32 arithmetic on them makes it
    (FP32 unit roundoff by default).  Returns the state after `steps` steps,
    or a list of states at the given checkpoints."""
    rng = np.random.default_rng(seed)
    f = f0.copy()
    out, want = [], set(checkpoints or [])
    for t in range(1, steps + 1):
        f = oracle.step(p, f)
        f *= 1.0 + rel * (2.0 * rng.random(f.shape) - 1.0)
        if t in want:
            out.append(f.copy())
    return out if checkpoints else f
