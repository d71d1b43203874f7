"""The oracle's Philox4x32-10 against an independent implementation: rocRAND's
host-side generator (ROCRAND_RNG_PSEUDO_PHILOX4_32_10, called through its C
API; it needs the HIP runtime, hence the gpu mark).  Its output stream with
seed S is, for output index s, word s & 3 of Philox(counter = (s >> 2 as a
64-bit value in the first two counter words, 0, 0), key = (S & 0xffffffff,
S >> 32)); rocrand_set_offset starts the stream at index offset.  Offsets
beyond 4 * 2^32 carry into the second counter word, where the oracle keeps the
sweep counter.  The same mapping holds under the default and legacy orderings.
"""
import ctypes
import os

import numpy as np
import pytest

from oracle import philox

pytestmark = pytest.mark.gpu

PHILOX4_32_10 = 404
ORDERINGS = {"default": 101, "legacy": 103}


def _rocrand(seed, offset, n, ordering):
    lib = ctypes.CDLL(os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "lib", "librocrand.so"))
    gen = ctypes.c_void_p()
    assert lib.rocrand_create_generator_host_blocking(ctypes.byref(gen), PHILOX4_32_10) == 0
    try:
        assert lib.rocrand_set_seed(gen, ctypes.c_ulonglong(seed)) == 0
        assert lib.rocrand_set_ordering(gen, ordering) == 0
        assert lib.rocrand_set_offset(gen, ctypes.c_ulonglong(offset)) == 0
        out = np.zeros(n, dtype=np.uint32)
        assert lib.rocrand_generate(gen, out.ctypes.data_as(ctypes.c_void_p), ctypes.c_size_t(n)) == 0
    finally:
        lib.rocrand_destroy_generator(gen)
    return out


def _oracle_stream(seed, offset, n):
    key = (seed & 0xffffffff, seed >> 32)
    out = []
    for s in range(offset, offset + n):
        c = s >> 2
        out.append(philox.philox4x32_10((c & 0xffffffff, (c >> 32) & 0xffffffff, 0, 0), key)[s & 3])
    return np.array(out, dtype=np.uint32)


@pytest.mark.parametrize("ordering", list(ORDERINGS))
@pytest.mark.parametrize("seed,offset", [(0x123456789ABCDEF0, 0), (0, 0), (2 ** 64 - 1, 1000),
                                         (16990, 4 * (2 ** 32 + 5) + 3), (987654321, 4 * (3 * 2 ** 32 - 2))])
def test_oracle_philox_equals_rocrand(seed, offset, ordering):
    n = 2048
    got = _rocrand(seed, offset, n, ORDERINGS[ordering])
    want = _oracle_stream(seed, offset, n)
    assert np.array_equal(got, want), (seed, offset, int(np.argmax(got != want)))
