"""Batched lattices, graph replay and launch variants through the C ABI.

A lattice advanced inside a batch, by replayed HIP graphs, or with any
tuning variant (segment height, prefetch, streaming stores) must produce the
same fields bit for bit as the plain single-lattice path: the per-site
arithmetic does not depend on tiling or launch mode.  Observable reductions
are fixed-order per lattice, so they agree bit for bit as well when the
lattice keeps its tiling.
"""
import numpy as np
import pytest
import torch  # noqa: F401  (first import can be slow; keep it out of test timeouts)

from paper_0906_3611_amd import inputs

pytestmark = pytest.mark.gpu

BASE = dict(tau=(1.0, 1.0), rho0=0.83, G_a=(-9.0, -9.0), G_r=(8.1, 8.1), G_AB=0.405)


def _lb():
    from paper_0906_3611_amd import lb
    return lb


def _specs(precision, boundary):
    u = 0.01 if boundary == "couette" else 0.0
    s = []
    for nx, ny, ga in ((67, 45, -9.0), (130, 70, -8.5), (64, 64, -9.3), (5, 9, -9.0)):
        d = dict(BASE)
        d.update(nx=nx, ny=ny, G_a=(ga, ga), precision=precision, boundary=boundary, u_wall=u)
        s.append(d)
    return s


def _fields_of(spec, seed):
    return inputs.noise_fields(spec["nx"], spec["ny"], seed, 0.5, 0.5, 0.05)


@pytest.mark.parametrize("precision", ["fp64", "fp32dev"])
@pytest.mark.parametrize("boundary", ["periodic", "couette"])
def test_batch_matches_single_bitwise(precision, boundary):
    lb = _lb()
    specs = _specs(precision, boundary)
    b = lb.Batch(specs)
    singles = []
    for i, sp in enumerate(specs):
        ra, rb = _fields_of(sp, 100 + i)
        b.init(i, ra, rb)
        kw = dict(sp)
        nx, ny = kw.pop("nx"), kw.pop("ny")
        lat = lb.Lattice(nx, ny, **kw)
        lat.init(ra, rb)
        singles.append(lat)
    b.step(13)
    for lat in singles:
        lat.step(13)
    obs_b = b.observables()
    for i, lat in enumerate(singles):
        assert np.array_equal(b.populations(i), lat.populations()), i
        o = lat.observables()
        assert np.array_equal(obs_b[i]["mass"], o["mass"]), i
        assert np.array_equal(obs_b[i]["mom"], o["mom"]), i
        assert obs_b[i]["pxy_kin"] == o["pxy_kin"], i
        assert np.array_equal(obs_b[i]["wall_stress"], o["wall_stress"]), i
        assert obs_b[i]["step"] == 13
    info = b.launch_info()
    assert info["ntiles"] >= sum(l.launch_info()["nstrips"] for l in singles)


def test_batch_rejects_mixed_precision_and_uninitialized_step():
    lb = _lb()
    specs = _specs("fp64", "periodic")
    specs[1] = dict(specs[1], precision="fp32dev")
    with pytest.raises(lb.LBError) as ei:
        lb.Batch(specs)
    assert ei.value.code == lb.LB_E_INVAL
    b = lb.Batch(_specs("fp64", "periodic"))
    b.init_noise(0, 1, 0.5, 0.5, 0.01)
    with pytest.raises(lb.LBError) as ei:
        b.step(1)
    assert ei.value.code == lb.LB_E_STATE


@pytest.mark.parametrize("precision", ["fp64", "fp32dev"])
def test_graph_replays_match_eager(precision):
    """Two-step graphs replayed several times, with eager work and
    synchronizations between the replays, against plain launches."""
    lb = _lb()
    nx, ny = 70, 48
    ra, rb = inputs.noise_fields(nx, ny, 3, 0.5, 0.5, 0.05)
    eager = lb.Lattice(nx, ny, precision=precision, **BASE)
    graph = lb.Lattice(nx, ny, precision=precision, **BASE)
    graph.set_launch(use_graph=1)
    assert graph.launch_info()["use_graph"] == 1
    for lat in (eager, graph):
        lat.init(ra, rb)
    for n in (2, 4, 3, 6, 1, 2):  # odd counts leave the graph parity changed
        eager.step(n)
        graph.step(n)
        o1, o2 = eager.observables(), graph.observables()  # eager work between replays
        assert np.array_equal(o1["mass"], o2["mass"])
        assert np.array_equal(eager.populations(), graph.populations()), n
    assert graph.t == eager.t == 18


def test_batch_graph_matches_batch_eager():
    lb = _lb()
    specs = _specs("fp32dev", "periodic")
    a, b = lb.Batch(specs), lb.Batch(specs)
    b.set_launch(use_graph=1)
    for i, sp in enumerate(specs):
        ra, rb = _fields_of(sp, 7 + i)
        a.init(i, ra, rb)
        b.init(i, ra, rb)
    for n in (4, 2, 5):
        a.step(n)
        b.step(n)
        for i in range(len(specs)):
            assert np.array_equal(a.populations(i), b.populations(i))


@pytest.mark.parametrize("precision", ["fp64", "fp32dev"])
def test_launch_variants_do_not_change_fields(precision):
    lb = _lb()
    nx, ny = 200, 96
    ra, rb = inputs.noise_fields(nx, ny, 9, 0.5, 0.5, 0.05)
    ref = lb.Lattice(nx, ny, precision=precision, **BASE)
    ref.init(ra, rb)
    ref.step(11)
    f_ref = ref.populations()
    for seg_h, pf, nt, grp in ((4, 0, 0, 1), (8, 1, 1, 1), (33, 0, 1, 4), (96, 1, 0, 4),
                               (16, 2, 1, 4), (12, 2, 0, 1), (7, 1, 1, 4)):
        lat = lb.Lattice(nx, ny, precision=precision, **BASE)
        lat.set_launch(seg_h=seg_h, prefetch=pf, stream_stores=nt, tiles_per_group=grp)
        info = lat.launch_info()
        assert (info["prefetch"], info["stream_stores"]) == (pf, nt)
        # 200 columns: 4 strips, so four tiles of a segment may share a workgroup
        g = grp if precision == "fp32dev" else 1
        assert info["tiles_per_group"] == g
        assert info["block_threads"] == (128 * g if precision == "fp32dev" else 64)
        assert info["grid_blocks"] == 8 * ((info["ntiles"] // g + 7) // 8)
        lat.init(ra, rb)
        lat.step(11)
        assert np.array_equal(lat.populations(), f_ref), (seg_h, pf, nt, grp)


@pytest.mark.parametrize("boundary", ["periodic", "couette"])
def test_autotune_leaves_the_evolution_unchanged(boundary):
    """lb_autotune times candidates on the live state, then restores it: the
    run continues exactly as if it had not been called."""
    lb = _lb()
    nx, ny = 200, 96
    u = 0.01 if boundary == "couette" else 0.0
    ra, rb = inputs.noise_fields(nx, ny, 12, 0.5, 0.5, 0.05)
    a = lb.Lattice(nx, ny, precision="fp32dev", boundary=boundary, u_wall=u, **BASE)
    b = lb.Lattice(nx, ny, precision="fp32dev", boundary=boundary, u_wall=u, **BASE)
    for lat in (a, b):
        lat.init(ra, rb)
        lat.step(7)
    res = b.autotune(steps=4)
    assert b.t == 7
    assert res["us_per_step"] > 0 and res["ntiles"] >= 1
    assert res["seg_h"] >= 1 and res["prefetch"] in (0, 1, 2) and res["stream_stores"] in (0, 1)
    a.step(9)
    b.step(9)
    assert np.array_equal(a.populations(), b.populations())
    oa, ob = a.observables(), b.observables()
    assert np.array_equal(oa["mass"], ob["mass"]) or np.allclose(oa["mass"], ob["mass"], rtol=1e-14)


def test_batch_autotune_leaves_the_evolution_unchanged():
    lb = _lb()
    specs = _specs("fp32dev", "periodic")
    a, b = lb.Batch(specs), lb.Batch(specs)
    b.set_launch(use_graph=1)
    for i, sp in enumerate(specs):
        ra, rb = _fields_of(sp, 40 + i)
        a.init(i, ra, rb)
        b.init(i, ra, rb)
    a.step(3)
    b.step(3)
    res = b.autotune(steps=4)
    assert res["us_per_step"] > 0 and res["use_graph"] == 1
    a.step(6)
    b.step(6)
    for i in range(len(specs)):
        assert np.array_equal(a.populations(i), b.populations(i)), i


def test_batch_common_segment_height():
    lb = _lb()
    specs = _specs("fp64", "couette")
    b = lb.Batch(specs)
    b.set_launch(seg_h=16)
    info = b.launch_info()
    assert info["seg_h"] <= 16  # 45 rows in 3 segments of 15
    singles = []
    for i, sp in enumerate(specs):
        ra, rb = _fields_of(sp, 60 + i)
        b.init(i, ra, rb)
        kw = dict(sp)
        nx, ny = kw.pop("nx"), kw.pop("ny")
        lat = lb.Lattice(nx, ny, **kw)
        lat.init(ra, rb)
        singles.append(lat)
    b.step(8)
    for i, lat in enumerate(singles):
        lat.step(8)
        assert np.array_equal(b.populations(i), lat.populations()), i


@pytest.mark.parametrize("precision", ["fp64", "fp32dev"])
def test_init_discs_equals_host_disc_fields(precision):
    """lb_init_discs builds the emulsion in the library; the state equals
    lb_init of the Python generator's densities bit for bit."""
    lb = _lb()
    nx, ny = 150, 70
    ra, rb = inputs.disc_fields(nx, ny, 21, 0.6)
    a = lb.Lattice(nx, ny, precision=precision, **BASE)
    b = lb.Lattice(nx, ny, precision=precision, **BASE)
    a.init(ra, rb)
    b.init_discs(21, 0.6)
    assert np.array_equal(a.populations(), b.populations())
    bt = lb.Batch([dict(BASE, nx=nx, ny=ny, precision=precision)] * 2)
    bt.init_discs(0, 21, 0.6)
    bt.init(1, ra, rb)
    assert np.array_equal(bt.populations(0), bt.populations(1))


def test_autotune_result_is_kept_per_shape():
    """A second lattice of the same shape, precision and boundary takes the
    kept result with steps = 0 (no timing) and keeps evolving exactly."""
    lb = _lb()
    nx, ny = 136, 80
    ra, rb = inputs.noise_fields(nx, ny, 31, 0.5, 0.5, 0.05)
    a = lb.Lattice(nx, ny, precision="fp32dev", **BASE)
    a.init(ra, rb)
    first = a.autotune(steps=4)
    b = lb.Lattice(nx, ny, precision="fp32dev", **BASE)
    b.init(ra, rb)
    again = b.autotune(steps=0)
    for k in ("seg_h", "prefetch", "stream_stores", "ntiles"):
        assert again[k] == first[k], k
    assert again["us_per_step"] == first["us_per_step"]
    a.step(5)
    b.step(5)
    assert np.array_equal(a.populations(), b.populations())


@pytest.mark.parametrize("precision", ["fp64", "fp32dev"])
def test_observables_do_not_depend_on_segment_height(precision):
    """Observables and wall averages are reduced over (row, strip) and strip
    partials, so re-cutting the segments mid-run changes nothing, bit for bit."""
    lb = _lb()
    nx, ny = 150, 100
    ra, rb = inputs.noise_fields(nx, ny, 5, 0.5, 0.5, 0.05)
    kw = dict(precision=precision, boundary="couette", u_wall=0.01, **BASE)
    a, b = lb.Lattice(nx, ny, **kw), lb.Lattice(nx, ny, **kw)
    a.set_launch(seg_h=8)
    for lat in (a, b):
        lat.init(ra, rb)
        lat.step(6)
    b.set_launch(seg_h=33)
    a.step(7)
    b.step(7)
    oa, ob = a.observables(), b.observables()
    for k in ("mass", "mom", "mom_phys", "wall_stress"):
        assert np.array_equal(oa[k], ob[k]), k
    assert oa["pxy_kin"] == ob["pxy_kin"] and oa["avg_count"] == ob["avg_count"] == 13


@pytest.mark.parametrize("precision", ["fp64", "fp32dev"])
def test_multi_chunk_observables_are_order_fixed(precision):
    """A lattice whose (row, strip) partials span several reduction chunks
    (2048 x 600: 19 200 slots, chunks of 8192, the last one partial) gives
    the same observables bit for bit alone, inside a batch, at another
    segment height and on a repeated call, and its mass matches the host's
    FP64 sum of the initial densities to round-off."""
    lb = _lb()
    nx, ny = 2048, 600
    ra, rb = inputs.noise_fields(nx, ny, 9, 0.5, 0.5, 0.05)
    kw = dict(precision=precision, boundary="couette", u_wall=0.01, **BASE)
    a, c = lb.Lattice(nx, ny, **kw), lb.Lattice(nx, ny, **kw)
    small = dict(BASE, nx=67, ny=45, precision=precision, boundary="couette", u_wall=0.01)
    bat = lb.Batch([dict(BASE, nx=nx, ny=ny, precision=precision, boundary="couette",
                         u_wall=0.01), small])
    c.set_launch(seg_h=24)
    for lat in (a, c):
        lat.init(ra, rb)
    bat.init(0, ra, rb)
    bat.init(1, *_fields_of(small, 7))
    for run in (a, c, bat):
        run.step(5)
    oa, oc, ob = a.observables(), c.observables(), bat.observables()[0]
    oa2 = a.observables()
    for o in (oc, ob, oa2):
        for k in ("mass", "mom", "mom_phys", "wall_stress"):
            assert np.array_equal(oa[k], o[k]), k
        assert oa["pxy_kin"] == o["pxy_kin"]
    mass0 = [float(np.sum(ra)), float(np.sum(rb))]
    for k in (0, 1):
        assert abs(oa["mass"][k] / mass0[k] - 1.0) < (1e-12 if precision == "fp64" else 1e-7), k


@pytest.mark.parametrize("precision,nx,ny,seg_h,grp,pf,nt", [
    ("fp32dev", 1024, 1024, 8, 1, 1, 0),     # ~2048 tiles: one wave of resident workgroups
    ("fp32dev", 4096, 1024, 32, 4, 0, 1),    # larger than the Infinity Cache: grouped tiles
    ("fp32dev-couette", 4096, 1024, 32, 4, 0, 1),
    ("fp32dev", 4096, 4096, 128, 4, 0, 1),   # taller segments keep the halo rows in L2
    ("fp32dev", 128, 128, 4, 1, 1, 0),       # too small to fill the GPU: shortest march
    ("fp64", 1024, 1024, 16, 1, 2, 0),       # ~1024 tiles; under twice the Infinity Cache
    ("fp64", 4096, 1024, 64, 1, 2, 1),
    ("fp64", 4096, 4096, 256, 1, 2, 1),
    ("fp32mom", 4096, 4096, 32, 1, 0, 1),    # issue-bound: at most 32-row segments
    ("fp32mom", 128, 128, 4, 1, 1, 0),
])
def test_default_tile_policy(precision, nx, ny, seg_h, grp, pf, nt):
    """The default launch shapes are the measured best ones (see the policy
    in lb_engine.hip); a change of the policy shows up here."""
    walls = dict(boundary="couette", u_wall=0.005) if precision.endswith("-couette") else {}
    lat = _lb().Lattice(nx, ny, precision=precision.split("-")[0], **walls, **BASE)
    info = lat.launch_info()
    assert info["seg_h"] == seg_h, info
    assert info["tiles_per_group"] == grp, info
    assert info["prefetch"] == pf, info
    assert info["stream_stores"] == nt, info
    assert info["ntiles"] == info["nstrips"] * info["nsegs"]
    lat.close()


def test_grouped_tiles_apply_only_where_every_lattice_allows_them():
    """Four tiles per workgroup need periodic lattices whose strip counts are
    all multiples of four; a batch of such lattices steps bit for bit as its
    members alone, other batches and walled lattices fall back to one tile,
    and a group size other than 1 or 4 is refused."""
    lb = _lb()
    shapes = [(256, 80), (512, 48), (252, 70)]   # 4, 8 and 4 strips
    specs = [dict(BASE, nx=nx, ny=ny, precision="fp32dev") for nx, ny in shapes]
    b = lb.Batch(specs)
    b.set_launch(tiles_per_group=4)
    assert b.launch_info()["tiles_per_group"] == 4
    singles = []
    for i, sp in enumerate(specs):
        ra, rb = _fields_of(sp, 40 + i)
        b.init(i, ra, rb)
        lat = lb.Lattice(sp["nx"], sp["ny"], precision="fp32dev", **BASE)
        lat.set_launch(tiles_per_group=1)
        lat.init(ra, rb)
        lat.step(9)
        singles.append(lat)
    b.step(9)
    for i, lat in enumerate(singles):
        assert np.array_equal(b.populations(i), lat.populations()), i
        assert np.array_equal(b.observables()[i]["mass"], lat.observables()["mass"]), i
    mixed = lb.Batch(specs + [dict(BASE, nx=320, ny=40, precision="fp32dev")])  # 5 strips
    mixed.set_launch(tiles_per_group=4)
    assert mixed.launch_info()["tiles_per_group"] == 1
    fp64 = lb.Lattice(256, 80, precision="fp64", **BASE)
    fp64.set_launch(tiles_per_group=4)
    assert fp64.launch_info()["tiles_per_group"] == 1
    with pytest.raises(RuntimeError):
        fp64.set_launch(tiles_per_group=3)


@pytest.mark.parametrize("nx,ny", [(256, 80), (250, 97)])
def test_grouped_tiles_with_walls_match_single_tiles(nx, ny):
    """Walls with four tiles per workgroup (each tile with its own wall
    momentum): populations, observables and the averaged wall stress are
    those of one tile per workgroup, bit for bit (250 columns: a ragged last
    strip; 97 rows: segments of unequal heights)."""
    lb = _lb()
    ra, rb = inputs.noise_fields(nx, ny, 13, 0.5, 0.5, 0.05)
    runs = []
    for g in (1, 4):
        lat = lb.Lattice(nx, ny, precision="fp32dev", boundary="couette", u_wall=0.01, **BASE)
        lat.set_launch(seg_h=8, tiles_per_group=g)
        assert lat.launch_info()["tiles_per_group"] == g
        lat.init(ra, rb)
        lat.step(13)
        runs.append((lat.populations(), lat.observables()))
    (fa, oa), (fb, ob) = runs
    assert np.array_equal(fa, fb)
    for k in ("mass", "mom", "mom_phys", "wall_stress"):
        assert np.array_equal(oa[k], ob[k]), k
    assert oa["pxy_kin"] == ob["pxy_kin"]


def test_autotune_result_persists_across_processes(tmp_path):
    """With lb_set_tune_cache, a tuned result written by one process is
    applied with steps = 0 (no timing) by another."""
    import json
    import os
    import subprocess
    import sys
    cache = tmp_path / "tune.txt"
    prog = r'''
import json, sys
sys.path.insert(0, sys.argv[1])
import torch
from paper_0906_3611_amd import inputs, lb
lb.set_tune_cache(sys.argv[2])
lat = lb.Lattice(100, 70, precision="fp32dev", tau=(1.0, 1.0), rho0=0.83, G_a=(-9.0, -9.0),
                 G_r=(8.1, 8.1), G_AB=0.405)
lat.init(*inputs.noise_fields(100, 70, 5, 0.5, 0.5, 0.01))
r = lat.autotune(steps=int(sys.argv[3]))
print(json.dumps({k: r[k] for k in ("seg_h", "nsegs", "prefetch", "stream_stores", "us_per_step")}))
'''
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

    def run(steps):
        out = subprocess.run([sys.executable, "-c", prog, root, str(cache), str(steps)],
                             capture_output=True, text=True, timeout=240)
        assert out.returncode == 0, out.stderr[-2000:]
        return json.loads(out.stdout.strip().splitlines()[-1])

    first = run(8)
    assert "/f32dev/periodic/launch/100x70 " in cache.read_text()
    second = run(0)
    assert second == first
