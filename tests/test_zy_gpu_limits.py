"""Size limits on the device: the largest state the library accepts (34
qubits; 128 GiB in complex64), checked by closed forms, and the rejection of
larger or malformed requests.  Named to run after the other GPU tests, so the
large allocations come last."""

import math
import sys

import numpy as np
import pytest

from workloads import ghz_circuit, make_gates, KIND_U, H

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no HIP device", allow_module_level=True)

from paper_2010_09746_amd import qsim as Q  # noqa: E402


def _say(msg):
    print(msg, file=sys.stderr, flush=True)


def test_largest_state_ghz_and_hadamards():
    """34 qubits, complex64 (128 GiB): GHZ through the pass form, then H on
    every qubit of |0...0> through the plain form; both have closed forms."""
    n = 34
    _say(f"limits: n={n} complex64 GHZ")
    torch.cuda.empty_cache()
    st = Q.State(n, "c64")
    st.run(ghz_circuit(n), form="pass", k_tile=11, max_swaps=16, pinned=3, perm_exec="relabel")
    idx = np.array([0, (1 << n) - 1, 1, 12345, (1 << n) - 2], dtype=np.uint64)
    a = st.amplitudes(idx)
    s = 1 / math.sqrt(2)
    assert abs(a[0] - s) < 1e-6 and abs(a[1] - s) < 1e-6
    assert np.abs(a[2:]).max() < 1e-7
    z = st.expect_z()
    assert np.abs(z).max() < 1e-6
    assert abs(st.norm() - 1) < 1e-5
    _say(f"limits: n={n} complex64 uniform superposition")
    st.set_basis(0)
    st.run(make_gates([(KIND_U, q, -1, H) for q in range(n)]), form="plain")
    a = st.amplitudes(np.array([0, 7, (1 << n) - 1], dtype=np.uint64))
    assert np.abs(a - 2.0 ** (-n / 2)).max() < 1e-9
    assert np.abs(st.expect_z()).max() < 1e-5
    st.close()
    del st
    torch.cuda.empty_cache()


def test_requests_beyond_the_limits_are_rejected():
    buf = torch.empty(1 << 20, dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream().cuda_stream
    with pytest.raises(Q.QsimError):
        Q.qs_state_create(35, "c64", 0, 0, stream)      # above the largest state
    with pytest.raises(Q.QsimError):
        Q.qs_state_create(17, "c128", buf.data_ptr(), buf.numel(), stream)   # buffer too small
    st = Q.State(8, "c128")
    with pytest.raises(Q.QsimError):
        st.apply_gates(make_gates([(KIND_U, 8, -1, H)]))   # qubit out of range
    with pytest.raises(Q.QsimError):
        st.permute([0, 1, 2, 3, 4, 5, 6, 6])               # not a permutation
    with pytest.raises(Q.QsimError):
        st.run(make_gates([(KIND_U, 0, -1, H)]), form="pass", k_tile=0)    # no local qubits
    # a tile size above n means the whole state is one tile
    st.set_basis(0)
    st.run(make_gates([(KIND_U, 0, -1, H)]), form="pass", k_tile=20)
    assert abs(st.amplitudes(np.array([1], dtype=np.uint64))[0] - 1 / math.sqrt(2)) < 1e-12
    st.close()
