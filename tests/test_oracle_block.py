"""The block method of parity_util.block_oracle (CPU): the oracle run on a
small periodic block cut around a node reproduces, at the block centre, the
node of the whole-grid run for as many steps as the block's reach allows.
This is what makes sampled parity checks of full-size grids exact."""
import numpy as np

from parity_util import block_oracle, workload


def test_block_centre_equals_whole_grid_run(oracle_lib):
    from paper_2201_06039_amd import workloads as W
    w = workload("multi_droplet_512", nx=40, ny=40, nz=40)
    a = dict(w["init"]); a.pop("kind")
    a.update(count=4, rmin=4.0, rmax=7.0)
    fields = W.multi_droplet(40, **a)
    steps = 3
    s = oracle_lib.Sim(**w["params"])
    s.init_fields(*fields)
    s.step(steps)
    full = s.rho_u_T()
    s.close()
    rho0 = fields[0]
    rng = np.random.default_rng(5)
    iface = np.argwhere((rho0 > 1.0) & (rho0 < 5.0))
    nodes = [tuple(v) for v in iface[rng.choice(len(iface), 6, replace=False)]]
    nodes += [(0, 0, 0), (39, 20, 0), (5, 39, 39)]  # the grid's periodic seams
    got = block_oracle(w, fields, nodes, steps)
    for c in range(5):
        ref = np.array([full[c][n] for n in nodes])
        np.testing.assert_array_equal(got[c], ref)
