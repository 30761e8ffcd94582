"""Distinct handles used concurrently (the ABI's threading contract).

A handle is not thread-safe, but distinct handles may be used at the same
time: on different HIP streams, from different host threads, with the
process-wide autotuner cache shared between them.  Each lattice must still
evolve exactly as a lone lattice on the default stream does.
"""
import threading

import numpy as np
import pytest
import torch

from paper_0906_3611_amd import inputs

pytestmark = pytest.mark.gpu

BASE = dict(tau=(1.0, 1.0), rho0=0.83, G_a=(-9.0, -9.0), G_r=(8.1, 8.1), G_AB=0.405)


def _lb():
    from paper_0906_3611_amd import lb
    return lb


def _reference(nx, ny, seed, steps, precision):
    lb = _lb()
    ra, rb = inputs.noise_fields(nx, ny, seed, 0.5, 0.5, 0.05)
    ref = lb.Lattice(nx, ny, precision=precision, **BASE)
    ref.init(ra, rb)
    ref.step(steps)
    return (ra, rb), ref.populations()


@pytest.mark.parametrize("precision", ["fp32dev", "fp64"])
def test_lattices_on_side_streams_match_the_default_stream(precision):
    lb = _lb()
    (ra, rb), f_ref = _reference(96, 80, 3, 40, precision)
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    lats = [lb.Lattice(96, 80, precision=precision, stream=s, **BASE) for s in streams]
    for lat in lats:
        lat.init(ra, rb)
    for _ in range(10):  # enqueue on both streams in turn
        for lat in lats:
            lat.step(4)
    for lat in lats:
        assert np.array_equal(lat.populations(), f_ref)


def test_library_owned_memory_on_the_null_stream():
    lb = _lb()
    (ra, rb), f_ref = _reference(70, 66, 5, 25, "fp32dev")
    lat = lb.Lattice(70, 66, precision="fp32dev", use_torch=False, **BASE)
    lat.init(ra, rb)
    lat.step(25)
    assert np.array_equal(lat.populations(), f_ref)


def test_handles_driven_from_separate_threads():
    """Four host threads, each with its own lattice and stream, step, tune
    and read back at the same time."""
    lb = _lb()
    shapes = [(128, 64, 11), (90, 70, 12), (128, 64, 13), (64, 100, 14)]
    refs = [_reference(nx, ny, seed, 30, "fp32dev") for nx, ny, seed in shapes]
    out = [None] * len(shapes)
    errors = []

    def run(k):
        try:
            nx, ny, _ = shapes[k]
            (ra, rb), _ = refs[k]
            stream = torch.cuda.Stream()
            with torch.cuda.stream(stream):
                lat = lb.Lattice(nx, ny, precision="fp32dev", stream=stream, **BASE)
                lat.init(ra, rb)
                lat.step(10)
                lat.autotune(steps=4)  # state and step count restored
                lat.step(20)
                out[k] = lat.populations()
        except Exception as e:  # reported by the main thread
            errors.append(e)

    threads = [threading.Thread(target=run, args=(k,)) for k in range(len(shapes))]
    for t in threads:
        t.start()
    for t in threads:
        t.join(timeout=120)
    assert not errors, errors
    for k, (_, f_ref) in enumerate(refs):
        assert out[k] is not None, k
        assert np.array_equal(out[k], f_ref), shapes[k]


def test_binding_works_without_importing_torch_first(tmp_path):
    """A program that imports only the binding (torch is pulled in by it
    before the library loads, so one HIP runtime serves both): a lattice on
    torch's workspace and stream steps and reports the same mass as the
    stored initial state."""
    import os
    import subprocess
    import sys
    prog = r'''
import json, sys
sys.path.insert(0, sys.argv[1])
from paper_0906_3611_amd import lb
lat = lb.Lattice(70, 45, precision="fp32dev", tau=(1.0, 1.0), rho0=0.83, G_a=(-9.0, -9.0),
                 G_r=(8.1, 8.1), G_AB=0.405)
lat.init_noise(5, 0.5, 0.5, 0.01)
m0 = list(lat.observables()["mass"])
lat.step(10)
print(json.dumps({"m0": m0, "m1": list(lat.observables()["mass"])}))
'''
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    out = subprocess.run([sys.executable, "-c", prog, root], capture_output=True, text=True,
                         timeout=240)
    assert out.returncode == 0, out.stderr[-2000:]
    import json
    r = json.loads(out.stdout.strip().splitlines()[-1])
    assert np.allclose(r["m1"], r["m0"], rtol=1e-7)
