"""The step kernels on a grid too large for the buffer-resource addressing
(collected last: it needs about 30 GB of host memory for the oracle)."""
import pytest

from parity_util import errors, run_gpu, run_oracle, workload

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12


def test_plain_pointer_path_on_a_large_wall_grid_fp64():
    """A grid whose copy halves exceed 4 GiB (FP64, 344 x 336 x 334 nodes,
    16.1 GB of populations) runs the kernels with plain global pointers
    instead of buffer resources; with the walls, the heated patch and gravity
    of the pool-boiling workload, one step against the oracle at the FP64 bar
    (the oracle needs about 30 GB of host memory for it)."""
    w = workload("pool_boiling_256x256x384", nx=344, ny=336, nz=334)
    nn = 344 * 336 * 334
    assert 14 * ((nn + 127) // 128 * 128) * 8 > 0xFFFFFFFF  # beyond the buffer-resource path
    print("plain-pointer path 344x336x334 f64 steps=1", flush=True)
    e = errors(run_gpu(w, 1, "f64"), run_oracle(w, 1))
    print(f"  errors {e}", flush=True)
    for k in ("rho", "u", "T"):
        assert e[k] <= FP64_TOL, (k, e)
