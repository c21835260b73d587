"""Checkpoint and restore through the C interface: a run of 3 sweeps saved,
restored into a freshly built handle and continued for 2 sweeps equals 5
uninterrupted sweeps bit for bit (energies and tensors); a state saved with the
centre inside the tree restores to the same effective Hamiltonian; a
checkpoint of another problem is refused."""
import numpy as np
import pytest

from problems import config_problem
from tests.gpu_util import gpu_matvec

pytestmark = pytest.mark.gpu


def _handle(p):
    from paper_2507_21236_amd import AttnHandle
    a = AttnHandle(p)
    a.init_state()
    return a


@pytest.mark.parametrize("key", ["ising4_m8", "ising8_m32"])
def test_resume_is_bit_identical(tmp_path, key):
    p = config_problem(key)
    ref = _handle(p)
    e_ref, _ = ref.sweep(5)
    a = _handle(p)
    e1, _ = a.sweep(3)
    path = str(tmp_path / "s3.ckpt")
    a.checkpoint(path)
    a.close()
    b = _handle(p)
    b.restore(path)
    assert np.array_equal(b.sweep_history(), e1)
    e2, _ = b.sweep(2)
    got = np.concatenate([e1, e2])
    assert np.array_equal(got, e_ref), (got - e_ref)
    assert np.array_equal(b.sweep_history(), e_ref)
    for n in range(ref.n_nodes):
        assert np.array_equal(ref.get_tensor(n), b.get_tensor(n)), n


def test_restore_with_centre_inside_the_tree(tmp_path):
    p = config_problem("ising8_m32")
    a = _handle(p)
    a.sweep(1)
    node = 20
    a.move_center(node)
    x = np.random.default_rng(3).standard_normal(a.node_info(node)[0])
    y_a = gpu_matvec(a, node, x)
    path = str(tmp_path / "mid.ckpt")
    a.checkpoint(path)
    b = _handle(p)
    b.restore(path)
    assert b.center == node
    y_b = gpu_matvec(b, node, x)
    assert np.array_equal(y_a, y_b)
    e_a, _ = a.sweep(1)
    e_b, _ = b.sweep(1)
    assert e_a[0] == e_b[0]


def test_restore_refuses_another_problem(tmp_path):
    from paper_2507_21236_amd import AttnError
    a = _handle(config_problem("ising4_m8"))
    path = str(tmp_path / "x.ckpt")
    a.checkpoint(path)
    b = _handle(config_problem("ising4_m8", h=2.5))
    with pytest.raises(AttnError) as e:
        b.restore(path)
    assert e.value.code == -13
    c = _handle(config_problem("ising4_m8", identity_de=True))
    with pytest.raises(AttnError) as e:
        c.restore(path)
    assert e.value.code == -13
