"""Plant plausible mistakes in the oracle and check that a pin catches each.

Every mutation is applied on the CPU by monkeypatching one oracle function
with a wrong variant (a dropped term, a wrong sign, a transposed operand, a
missing scale); the listed pin from test_oracle_rsvd must then fail.
"""

import numpy as np
import pytest

from oracle import rsvd
from tests import test_oracle_rsvd as pins


def _no_power_steps(A, Omega, q):
    Q, _ = rsvd.qr_pos(A @ Omega)
    return Q


def _transposed_adjoint(A, Omega, q):
    Q, _ = rsvd.qr_pos(A @ Omega)
    for _ in range(q):
        Qt, _ = rsvd.qr_pos(A @ Q)           # A instead of A*
        Q, _ = rsvd.qr_pos(A @ Qt)
    return Q


def _fft_wrong_sign(A, d, R):
    n = A.shape[1]
    X = np.fft.ifft(A * d[None, :], axis=1) * n
    return X[:, np.asarray(R)] / np.sqrt(len(R))


def _fft_missing_scale(A, d, R):
    X = np.fft.fft(A * d[None, :], axis=1)
    return X[:, np.asarray(R)]


def _qr_unsigned(Y):
    return np.linalg.qr(Y, mode="reduced")


def _svd_forgets_adjoint(A, Q):
    B = rsvd.adj(Q) @ A
    Ut, S, Vh = np.linalg.svd(B, full_matrices=False)
    return Q @ Ut, S, Vh[: Vh.shape[0]].T[:, ::-1], B


def _truncate_wrong_end(U, S, V, k):
    return U[:, -k:], S[-k:], V[:, -k:]


def _srft_drops_signs(A, d, R):
    X = np.fft.fft(A, axis=1)
    return X[:, np.asarray(R)] / np.sqrt(len(R))


def _real_srft_wrong_pair(A, d, R):
    # sine and cosine columns swapped
    n = A.shape[1]
    l = len(R)
    X = np.fft.fft(A * d[None, :], axis=1)
    Y = np.empty((A.shape[0], l))
    for t, q in enumerate(np.asarray(R)):
        if q == 0 or 2 * q == n:
            Y[:, t] = X[:, q % n].real / np.sqrt(l)
        elif 2 * q < n:
            Y[:, t] = -np.sqrt(2.0 / l) * X[:, q].imag
        else:
            Y[:, t] = np.sqrt(2.0 / l) * X[:, n - q].real
    return Y


MUTATIONS = [
    ("real_srft_sketch", _real_srft_wrong_pair, pins.test_real_srft_sketch_equals_definition, {"n": 32, "l": 6}),
    ("randomized_subspace_iteration", _no_power_steps, pins.test_power_scheme_theorem_9_2, {"q": 1}),
    ("randomized_subspace_iteration", _transposed_adjoint,
     pins.test_subspace_iteration_spans_power_iteration, {"m": 90, "n": 90}),
    ("srft_sketch", _fft_wrong_sign, pins.test_srft_sketch_equals_definition, {}),
    ("srft_sketch", _fft_missing_scale, pins.test_srft_sketch_equals_definition, {}),
    ("srft_sketch", _srft_drops_signs, pins.test_srft_sketch_equals_definition, {}),
    ("qr_pos", _qr_unsigned, pins.test_qr_pos_is_a_qr, {}),
    ("direct_svd", _svd_forgets_adjoint, pins.test_full_sample_count_gives_exact_svd,
     {"m": 12, "n": 8, "q": 0}),
    ("truncate", _truncate_wrong_end, pins.test_exact_rank_recovery, {"q": 0}),
]


@pytest.mark.parametrize("name,bad,pin,kwargs", MUTATIONS,
                         ids=[f"{m[0]}:{m[1].__name__}" for m in MUTATIONS])
def test_pin_catches_mutation(monkeypatch, name, bad, pin, kwargs):
    pin(**kwargs)  # the pin passes on the real oracle
    monkeypatch.setattr(rsvd, name, bad)
    with pytest.raises((AssertionError, ValueError, np.linalg.LinAlgError)):
        pin(**kwargs)
