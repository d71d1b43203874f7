"""The C-ABI library loads, exports every symbol include/ising.h declares, and
rejects invalid arguments on the host (no device call is made by these)."""
import ctypes
import math
import os
import re

import pytest

import paper_2404_16990_amd as P

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = []
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            text = open(os.path.join(ROOT, "include", fn)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names += re.findall(r"\b(ising(?:3d)?_\w+)\s*\(", text)
    return sorted(set(names))


def test_header_declares_the_boundary():
    d = _declared()
    for required in ["ising_state_bytes", "ising_batch_create", "ising_batch_run",
                     "ising_batch_observables", "ising_batch_get_spins", "ising_batch_set_spins",
                     "ising_batch_destroy"]:
        assert required in d


def test_library_exports_every_declared_symbol():
    L = P.lib()
    for name in _declared():
        assert hasattr(L, name), name
    assert sorted(P.EXPORTED) == _declared()


def test_binding_has_the_same_names():
    for name in _declared():
        assert callable(getattr(P, name)), name


def _d(**kw):
    base = dict(Lx=64, Ly=64, J=1.0, beta=0.44, seed=1, replica=0, init=0)
    base.update(kw)
    return base


def test_state_bytes_layout():
    one = P.ising_state_bytes([_d()])
    two = P.ising_state_bytes([_d(), _d(Lx=128, Ly=6)])
    assert one >= 2 * 64 * 64 // 8 and two > one and two % 256 == 0


@pytest.mark.parametrize("kw,code", [
    (dict(Lx=100), P.ISING_E_UNSUPPORTED), (dict(Lx=0), P.ISING_E_UNSUPPORTED),
    (dict(Ly=7), P.ISING_E_UNSUPPORTED), (dict(Ly=0), P.ISING_E_UNSUPPORTED),
    (dict(J=0.0), P.ISING_E_INVALID), (dict(J=-1.0), P.ISING_E_INVALID),
    (dict(J=math.inf), P.ISING_E_INVALID), (dict(beta=-0.1), P.ISING_E_INVALID),
    (dict(beta=math.nan), P.ISING_E_INVALID), (dict(init=7), P.ISING_E_INVALID),
    (dict(rng=2), P.ISING_E_INVALID), (dict(rng=-1), P.ISING_E_INVALID),
])
def test_invalid_descriptors(kw, code):
    with pytest.raises(P.IsingError) as e:
        P.ising_state_bytes([_d(**kw)])
    assert e.value.code == code
    assert P.ising_last_error() != ""


def test_infinite_beta_is_valid():
    assert P.ising_state_bytes([_d(beta=math.inf)]) > 0


def test_both_random_number_contracts_are_valid():
    assert P.ising_state_bytes([_d(rng=P.ISING_RNG_SITE), _d(rng=P.ISING_RNG_BITSLICED)]) > 0
    assert P.ctypes.sizeof(P.ising_desc) == 48  # C layout: 40 bytes + int32 rng, 8-byte aligned


def test_create_rejects_before_touching_the_device():
    with pytest.raises(P.IsingError) as e:
        P.ising_batch_create([_d()], None, 1 << 20)
    assert e.value.code == P.ISING_E_INVALID
    with pytest.raises(P.IsingError) as e:
        P.ising_batch_create([_d()], 256, 16)  # too small
    assert e.value.code == P.ISING_E_NOMEM
    with pytest.raises(P.IsingError) as e:
        P.ising_batch_create([_d()], 0x1001, 1 << 20)  # misaligned
    assert e.value.code == P.ISING_E_INVALID
    with pytest.raises(P.IsingError) as e:
        P.ising_batch_create([], 256, 1 << 20)
    assert e.value.code == P.ISING_E_INVALID


def test_null_handles_are_rejected():
    for fn, args in [(P.lib().ising_batch_run, (None, 10, 0, None, None, None)),
                     (P.lib().ising_batch_observables, (None, None, None, None)),
                     (P.lib().ising_batch_get_spins, (None, 0, None, None))]:
        assert fn(*args) == P.ISING_E_INVALID
    assert P.lib().ising_batch_destroy(None) == P.ISING_OK


def test_strerror_covers_codes():
    for c in (0, -1, -2, -3, -4, -5):
        assert P.ising_strerror(c)


def test_nn_sizes_and_validation():
    assert P.ising_nn_param_count(64) == 62337
    with pytest.raises(P.IsingError) as e:
        P.ising_nn_param_count(32)
    assert e.value.code == P.ISING_E_UNSUPPORTED
    b8 = P.ising_nn_state_bytes(8, 64, 512, 65536)
    b2 = P.ising_nn_state_bytes(2, 64, 512, 65536)
    assert b8 > b2 > 0 and b8 % 256 == 0
    for args, code in [((3, 64, 16, 16), P.ISING_E_UNSUPPORTED), ((8, 48, 16, 16), P.ISING_E_UNSUPPORTED),
                       ((8, 64, 0, 16), P.ISING_E_INVALID), ((8, 64, 16, 1), P.ISING_E_INVALID)]:
        with pytest.raises(P.IsingError) as e:
            P.ising_nn_state_bytes(*args)
        assert e.value.code == code


def test_nn_create_rejects_before_touching_the_device():
    import numpy as np
    params = np.zeros(62337, dtype=np.float32)
    with pytest.raises(P.IsingError) as e:
        P.ising_nn_create(8, 64, 16, 16, params.ctypes.data, None, 1 << 30)
    assert e.value.code == P.ISING_E_INVALID
    with pytest.raises(P.IsingError) as e:
        P.ising_nn_create(8, 64, 16, 16, params.ctypes.data, 256, 16)
    assert e.value.code == P.ISING_E_NOMEM
    with pytest.raises(P.IsingError) as e:
        P.ising_nn_create(5, 64, 16, 16, params.ctypes.data, 256, 1 << 30)
    assert e.value.code == P.ISING_E_UNSUPPORTED
    for fn, args in [(P.lib().ising_nn_train_step, (None, None, None, None, 1, 1e-3, None, None)),
                     (P.lib().ising_nn_train_step_sampled, (None, None, None, None, 10, 1, 1e-3, 0, None, None)),
                     (P.lib().ising_nn_score, (None, 1, None, None, None, None, None)),
                     (P.lib().ising_batch_block_round, (None, None, 0, None, None))]:
        assert fn(*args) == P.ISING_E_INVALID
    assert P.lib().ising_nn_destroy(None) == P.ISING_OK


def _d3(**kw):
    base = dict(Lx=64, Ly=4, Lz=6, J=1.0, beta=0.22, seed=1, replica=0, init=0)
    base.update(kw)
    return base


def test_3d_layout_and_validation():
    assert P.ctypes.sizeof(P.ising3d_desc) == 48  # 4 int32, 3 x 8 bytes, 2 x 4 bytes
    one = P.ising3d_state_bytes([_d3()])
    assert one >= 2 * 64 * 4 * 6 // 8 and one % 256 == 0
    assert P.ising3d_state_bytes([_d3(), _d3(Lx=128, Lz=2), _d3(rng=P.ISING_RNG_BITSLICED)]) > one
    for kw, code in [(dict(Lx=96), P.ISING_E_UNSUPPORTED), (dict(Ly=3), P.ISING_E_UNSUPPORTED),
                     (dict(Lz=0), P.ISING_E_UNSUPPORTED), (dict(Lz=5), P.ISING_E_UNSUPPORTED),
                     (dict(Lx=65536, Ly=256, Lz=256), P.ISING_E_UNSUPPORTED),
                     (dict(J=0.0), P.ISING_E_INVALID), (dict(beta=-1.0), P.ISING_E_INVALID),
                     (dict(init=5), P.ISING_E_INVALID), (dict(rng=2), P.ISING_E_INVALID),
                     (dict(rng=-1), P.ISING_E_INVALID)]:
        with pytest.raises(P.IsingError) as e:
            P.ising3d_state_bytes([_d3(**kw)])
        assert e.value.code == code, kw
    with pytest.raises(P.IsingError) as e:
        P.ising3d_batch_create([_d3()], None, 1 << 20)
    assert e.value.code == P.ISING_E_INVALID
    with pytest.raises(P.IsingError) as e:
        P.ising3d_batch_create([_d3()], 256, 16)
    assert e.value.code == P.ISING_E_NOMEM
    for fn, args in [(P.lib().ising3d_batch_run, (None, 1, 0, None, None, None)),
                     (P.lib().ising3d_batch_observables, (None, None, None, None)),
                     (P.lib().ising3d_batch_get_spins, (None, 0, None, None))]:
        assert fn(*args) == P.ISING_E_INVALID
    assert P.lib().ising3d_batch_destroy(None) == P.ISING_OK
