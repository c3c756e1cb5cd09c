"""Batches of independent lattices (one persistent launch per step, graph
replays of two steps): every lattice of a batch must equal its stand-alone
run bit for bit, through graph replays, direct launches, the autotuner and
the null stream; and an FP64 batch must match the oracle."""
import copy

import numpy as np
import pytest

from parity_util import errors, run_oracle, workload
from paper_2201_06039_amd import workloads as W

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


def small_cases():
    """Uneven lattices: cubes and ragged boxes, static and evaporating
    droplets, one with the reservoir boundary."""
    out = []
    evap = W.load("evaporation_128")
    for (nx, ny, nz), R, hot, shell in [((24, 24, 24), 6.0, False, False),
                                        ((30, 26, 22), 6.5, True, False),
                                        ((40, 40, 40), 9.0, True, False),
                                        ((17, 33, 28), 5.0, False, False),
                                        ((26, 22, 20), 6.0, True, True),
                                        ((48, 48, 48), 11.0, False, False)]:
        w = copy.deepcopy(evap)
        w["params"].update(nx=nx, ny=ny, nz=nz)
        w["init"].update(radius=R, center=[nx / 2 - 0.3, ny / 2 + 0.2, nz / 2 - 0.1], seed=len(out))
        if not hot:
            w["init"]["T_v"] = w["init"]["T_l"]
        if shell:
            w["params"].update(bc_T_shell=1, T_shell=w["init"]["T_v"])
        out.append(w)
    return out


def solo(w, storage, schedule):
    from paper_2201_06039_amd import lbm
    lat = lbm.Lattice(w["params"], storage=storage, device="cuda:0")
    lat.init_fields(*W.fields(w))
    outs = []
    for n in schedule:
        lat.step(n)
        outs.append(lat.rho_u_T())
    lat.close()
    return outs


def make_batch(cases, storage, stream=None):
    from paper_2201_06039_amd import lbm
    b = lbm.Batch([w["params"] for w in cases], storage=storage, device="cuda:0", stream=stream)
    for c, w in enumerate(cases):
        b.init_case(c, *W.fields(w))
    return b


SCHEDULE = [1, 4, 3, 2]  # a direct launch, two graph replays, a replay and a direct launch, one replay


@pytest.mark.parametrize("storage", ["f16", "f32"])
def test_batch_equals_solo_runs(storage):
    cases = small_cases()
    b = make_batch(cases, storage)
    _say(f"batch {storage}: launch {b.launch()}")
    ref = [solo(w, storage, SCHEDULE) for w in cases]
    for k, n in enumerate(SCHEDULE):
        b.step(n)
        for c in range(len(cases)):
            got = b.rho_u_T(c)
            for x, y in zip(got, ref[c][k]):
                assert np.array_equal(x, y), (storage, k, c)
        _say(f"  after {sum(SCHEDULE[:k + 1])} steps: all {len(cases)} lattices bitwise equal to their solo runs")
    b.close()


@pytest.mark.parametrize("launch", [(32, 8, 8, 0), (64, 8, 32, 7), (128, 4, 4, 1), (32, 16, 16, 1000),
                                    (0, 0, 16, 0), (0, 0, 64, 3)])
def test_batch_launch_shapes(launch):
    """Tile, chunk and persistent-grid size (one workgroup included) change
    nothing in the results."""
    cases = small_cases()[:4]
    b = make_batch(cases, "f16")
    b.set_launch(*launch)
    _say(f"batch launch {b.launch()}")
    ref = [solo(w, "f16", [5]) for w in cases]
    b.step(5)
    for c in range(len(cases)):
        for x, y in zip(b.rho_u_T(c), ref[c][0]):
            assert np.array_equal(x, y), (launch, c)
    b.close()


def test_fitted_tiles():
    """Fitted tiles (launch tile 0 x 0): every lattice gets its own tile of
    256..512 nodes, exactly as wide as the lattice (whole rows, whose x halo
    comes from the tile's own columns) or 4k wide, whose extended tile fits
    the LDS ring of 700 nodes, leaving no more idle thread slots than the
    32 x 16 tile; the lattices still equal their solo runs bit for bit (FP32
    and FP16).  The cases cover whole rows of odd and even width, and a
    lattice wider than 128 with 4k-wide tiles ragged in x and y."""
    import math
    cases = small_cases()
    evap = W.load("evaporation_128")
    for k, (nx, ny, nz) in enumerate(((85, 20, 12), (150, 9, 10))):
        w = copy.deepcopy(evap)
        w["params"].update(nx=nx, ny=ny, nz=nz)
        w["init"].update(radius=3.0, center=[nx / 3, ny / 2, nz / 2], seed=40 + k)
        cases.append(w)
    for storage in ("f32", "f16"):
        b = make_batch(cases, storage)
        b.set_launch(0, 0, 32, 0)
        for c, w in enumerate(cases):
            tx, ty, thr = b.case_tile(c)
            nx, ny = w["params"]["nx"], w["params"]["ny"]
            assert thr == 512 and (tx == nx or tx % 4 == 0) and 256 <= tx * ty <= 512, (tx, ty)
            assert (tx + 2) * (ty + 2) <= 700, (tx, ty)
            assert math.ceil(nx / tx) * math.ceil(ny / ty) * 512 <= math.ceil(nx / 32) * math.ceil(ny / 16) * 512
            _say(f"  {storage} lattice {c} ({nx}x{ny}): tile {tx}x{ty}")
        ref = [solo(w, storage, [3])[0] for w in cases]
        b.step(3)
        for c in range(len(cases)):
            for x, y in zip(b.rho_u_T(c), ref[c]):
                assert np.array_equal(x, y), (storage, c)
        b.close()


def test_autotune_leaves_the_state_unchanged():
    cases = small_cases()
    b = make_batch(cases, "f16")
    b.step(3)
    ms = b.autotune(steps=2)
    _say(f"autotune: {ms:.4f} ms/step with {b.launch()}")
    assert ms > 0
    b.step(4)
    ref = [solo(w, "f16", [7]) for w in cases]
    for c in range(len(cases)):
        for x, y in zip(b.rho_u_T(c), ref[c][0]):
            assert np.array_equal(x, y), c
    b.close()


def test_batch_on_the_null_stream():
    """Without a stream of its own the batch launches directly (no graphs)."""
    import torch
    cases = small_cases()[:3]
    b = make_batch(cases, "f16", stream=torch.cuda.default_stream())
    ref = [solo(w, "f16", [4]) for w in cases]
    b.step(4)
    for c in range(len(cases)):
        for x, y in zip(b.rho_u_T(c), ref[c][0]):
            assert np.array_equal(x, y), c
    b.close()


def test_fp64_batch_against_oracle():
    cases = [workload("static_droplet_32", nx=20, ny=18, nz=16, radius=5.0),
             workload("evaporation_128", nx=24, ny=24, nz=24, radius=6.0),
             workload("d2_law_48", nx=22, ny=20, nz=18, radius=5.0)]
    b = make_batch(cases, "f64")
    b.step(30)
    for c, w in enumerate(cases):
        e = errors(b.rho_u_T(c), run_oracle(w, 30))
        _say(f"  case {c}: {e}")
        assert e["rho"] <= 1e-12 and e["T"] <= 1e-12 and e["u"] <= 1e-12, (c, e)
    b.close()


@pytest.mark.parametrize("storage", ["f16", "bf16", "f32"])
def test_batch_against_oracle(storage):
    """The batch in the reduced formats against the FP64 oracle directly
    (fitted tiles, uneven lattices of the benchmark's kinds, 30 steps): FP32
    at the single-lattice FP32 bar for rho and T, FP16 and BF16 within one
    rounding of the field in the storage type (2^-11, 2^-8) for rho and T and
    20 such roundings for u in the L2 sense, as for single lattices."""
    cases = [workload("static_droplet_32", nx=20, ny=18, nz=16, radius=5.0),
             workload("evaporation_128", nx=24, ny=24, nz=24, radius=6.0),
             workload("d2_law_48", nx=22, ny=20, nz=18, radius=5.0)]
    b = make_batch(cases, storage)
    b.set_launch(0, 0, 32, 0)
    b.step(30)
    tol = {"f32": 1e-5, "f16": 2.0 ** -11, "bf16": 2.0 ** -8}[storage]
    for c, w in enumerate(cases):
        e = errors(b.rho_u_T(c), run_oracle(w, 30))
        _say(f"  {storage} case {c} (tile {b.case_tile(c)[:2]}): {e}")
        assert e["rho"] <= tol and e["T"] <= tol, (c, e)
        if storage != "f32":
            assert e["u_l2"] <= 20 * tol, (c, e)
    b.close()


def test_batch_reduce_and_readout_errors():
    from paper_2201_06039_amd import lbm
    cases = small_cases()[:2]
    b = lbm.Batch([w["params"] for w in cases], storage="f16", device="cuda:0")
    with pytest.raises(lbm.LbmError) as ei:
        b.step(1)  # nothing initialised yet
    assert ei.value.status == lbm.ESTATE
    for c, w in enumerate(cases):
        b.init_case(c, *W.fields(w))
    m0 = [b.reduce(c)[0] for c in range(2)]
    b.step(10)
    m1 = [b.reduce(c)[0] for c in range(2)]
    for a, z in zip(m0, m1):
        assert abs(z - a) / a < 1e-5
    assert b.lib.lbm_batch_get_rho_u_T(b._h, 5, None, None, None, None, None) == lbm.EINVAL
    assert b.lib.lbm_batch_set_launch(b._h, 48, 8, 16, 0) == lbm.EINVAL
    b.close()


def test_full_batch_256_sampled_cases_equal_solo_runs():
    """The benchmark's batch (256 lattices, 74.5 M nodes, FP16) in its
    autotuned launch: after 20 steps (graph replays) the smallest, the largest
    and two more lattices equal their stand-alone runs bit for bit, and no
    lattice is unstable."""
    from paper_2201_06039_amd import lbm
    wb = W.load("batch_256")
    cases = wb["cases"]
    b = lbm.Batch([c["params"] for c in cases], storage="f16", device="cuda:0")
    for i, c in enumerate(cases):
        b.init_case(i, *W.fields(c))
    ms = b.autotune(steps=3)
    _say(f"batch_256: autotuned {b.launch()} at {ms:.3f} ms/step")
    b.step(20)
    sizes = [c["params"]["nx"] for c in cases]
    picks = sorted({int(np.argmin(sizes)), int(np.argmax(sizes)), 17, 200})
    for i in range(len(cases)):
        b.reduce(i)  # raises on an unstable lattice
    for i in picks:
        tile = b.launch()
        ref = solo(cases[i], "f16", [20])[0]
        for x, y in zip(b.rho_u_T(i), ref):
            assert np.array_equal(x, y), (i, tile)
        _say(f"  lattice {i} (L = {sizes[i]}) bitwise equal to its solo run")
    b.close()
