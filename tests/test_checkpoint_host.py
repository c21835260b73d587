"""Host-side tests of the checkpoint format (no GPU): the problem hash a
handle records, and the header reader on files written here byte by byte in
the documented layout (magic, version, byte-order marker, hash, sizes,
disentanglers, centre, isometry directions, sweep energies, tensors, FNV-1a
checksum of everything before it)."""
import struct

import numpy as np
import pytest

from problems import config_problem
from paper_2507_21236_amd import AttnHandle, ATTN_HOST_ONLY, AttnError
from paper_2507_21236_amd import _lib


def _fnv(data):
    v = 1469598103934665603
    for c in data:
        v ^= c
        v = (v * 1099511628211) & 0xFFFFFFFFFFFFFFFF
    return v


def _file(hash_, n_nodes=3, center=2, energies=(-1.5, -2.5), tensors=(0.5, 0.25), n_de=1, d=2):
    body = b"ATTNCKPT" + struct.pack("<II", 1, 0x01020304) + struct.pack("<Q", hash_)
    body += struct.pack("<4i", 4, d, 8, n_nodes)
    body += struct.pack("<i", n_de) + np.eye(d * d).ravel().tobytes() * n_de
    body += struct.pack("<i", center) + struct.pack(f"<{n_nodes}i", *([2] * n_nodes))
    body += struct.pack("<q", len(energies)) + np.asarray(energies, dtype=np.float64).tobytes()
    body += struct.pack("<q", len(tensors)) + np.asarray(tensors, dtype=np.float64).tobytes()
    return body + struct.pack("<Q", _fnv(body))


def test_problem_hash_tracks_the_hamiltonian_not_the_gates():
    p = config_problem("ising4_m8")
    h1 = AttnHandle(p, flags=ATTN_HOST_ONLY).problem_hash()
    assert h1 == AttnHandle(config_problem("ising4_m8"), flags=ATTN_HOST_ONLY).problem_hash()
    # another field: different hash
    assert h1 != AttnHandle(config_problem("ising4_m8", h=3.1), flags=ATTN_HOST_ONLY).problem_hash()
    q = config_problem("ising4_m8", m=4)
    assert h1 != AttnHandle(q, flags=ATTN_HOST_ONLY).problem_hash()
    # other disentangler matrices on the same sites: same hash (the file records them)
    r = config_problem("ising4_m8", identity_de=True)
    assert r.de_sites == p.de_sites
    assert h1 == AttnHandle(r, flags=ATTN_HOST_ONLY).problem_hash()


def test_checkpoint_header_reader(tmp_path):
    f = tmp_path / "a.ckpt"
    f.write_bytes(_file(0x1234ABCD5678EF01))
    assert _lib.attn_checkpoint_info(str(f)) == (0x1234ABCD5678EF01, 3, 2, 2)


@pytest.mark.parametrize("damage", ["truncate", "flip", "magic", "empty"])
def test_checkpoint_reader_rejects_damaged_files(tmp_path, damage):
    data = bytearray(_file(42))
    if damage == "truncate":
        data = data[:-20]
    elif damage == "flip":
        data[60] ^= 1
    elif damage == "magic":
        data[0:8] = b"NOTACKPT"
    else:
        data = bytearray()
    f = tmp_path / "b.ckpt"
    f.write_bytes(bytes(data))
    with pytest.raises(AttnError) as e:
        _lib.attn_checkpoint_info(str(f))
    assert e.value.code == -12                       # ATTN_ERR_IO


def test_checkpoint_calls_need_a_device_state(tmp_path):
    a = AttnHandle(config_problem("ising4_m8"), flags=ATTN_HOST_ONLY)
    with pytest.raises(AttnError) as e:
        a.checkpoint(str(tmp_path / "c.ckpt"))
    assert e.value.code == -8                        # STATE: host-only handle
    with pytest.raises(AttnError) as e:
        _lib.attn_checkpoint_info(str(tmp_path / "missing.ckpt"))
    assert e.value.code == -12
    assert len(a.sweep_history()) == 0
