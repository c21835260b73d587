"""FP64 Lanczos sweeps replayed from HIP graphs (attn_sweep_opts.use_graphs)
against the same sweeps launched one kernel at a time, through the C
interface: energies, tensors, counters and matvecs in between must agree bit
for bit, over several replays of each graph with the program's own eager work
and synchronisations between them."""
import numpy as np
import pytest

from problems import config_problem

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _matvec(a, x):
    import torch
    n = a.center
    xt = torch.from_numpy(np.ascontiguousarray(x)).to("cuda")
    yt = torch.empty_like(xt)
    a.heff_apply(n, xt, yt)
    torch.cuda.synchronize()
    return yt.cpu().numpy()


@pytest.mark.parametrize("key", ["ising4_m8", "ising8_m16"])
def test_graph_sweeps_reproduce_eager_sweeps(key):
    from paper_2507_21236_amd import AttnHandle
    p = config_problem(key)
    ag, ae = AttnHandle(p), AttnHandle(p)   # replayed from graphs / eager
    rng = np.random.default_rng(11)
    for rnd in range(2):   # the second round starts from a fresh state again: cached graph
        ag.init_state()
        ae.init_state()
        for s in range(4):
            eg, _ = ag.sweep(1, use_graphs=True)
            ee, _ = ae.sweep(1)
            assert eg[0] == ee[0], (rnd, s, eg[0], ee[0])
            assert ag.center == ae.center
            # eager work on the same device between the replays
            x = rng.standard_normal(ag.get_tensor(ag.center).shape)
            assert np.array_equal(_matvec(ag, x), _matvec(ae, x)), (rnd, s)
        for n in range(ag.n_nodes):
            assert np.array_equal(ag.get_tensor(n), ae.get_tensor(n)), (rnd, n)
        assert ag.counters() == ae.counters()
    # a sweep without graphs on the graph handle continues the same trajectory
    eg, _ = ag.sweep(1)
    ee, _ = ae.sweep(1)
    assert eg[0] == ee[0]
