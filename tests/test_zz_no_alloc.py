"""lbm_reduce_static, the allocation-free variant of lbm_reduce (its scratch
is a static device array of the library), through the C-ABI: on two calls in
a row, the second on a smaller grid, it must give lbm_reduce's results bit
for bit (same kernels, same summation order), and a grid beyond its scratch
is refused with ESCRATCH."""
import pytest

from parity_util import workload

pytestmark = pytest.mark.gpu


def test_reduce_static_matches_reduce_on_two_calls():
    from paper_2201_06039_amd import lbm, workloads as W
    cases = [("f16", workload("evaporation_128", nx=96, ny=80, nz=64, radius=18.0), 7),
             ("f32", workload("static_droplet_32", nx=24, ny=20, nz=18, radius=5.0), 5)]
    for storage, w, steps in cases:
        p = w["params"]
        print(f"reduce_static {storage} {p['nx']}x{p['ny']}x{p['nz']}", flush=True)
        lat = lbm.Lattice(p, storage=storage, device="cuda:0")
        lat.init_fields(*W.fields(w))
        lat.step(steps)
        ref = lat.reduce()
        got = lat.reduce_static()
        lat.close()
        assert got == ref, (storage, got, ref)
        assert ref[0] > 0 and ref[1] > 0


def test_reduce_static_refuses_grids_beyond_its_scratch():
    from paper_2201_06039_amd import lbm
    w = workload("static_droplet_32", nx=1024, ny=512, nz=520)  # 272,629,760 nodes > 268,434,432
    lat = lbm.Lattice(w["params"], storage="f16", device="cuda:0")
    with pytest.raises(lbm.LbmError) as err:
        lat.reduce_static()
    assert err.value.status == lbm.ESCRATCH
    lat.close()
