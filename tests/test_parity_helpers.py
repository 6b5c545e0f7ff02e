"""The GPU parity gate itself (CPU): a non-finite output must fail it."""
import numpy as np

from _parity import error_report, gate


def test_gate_rejects_nan_and_inf():
    ref = np.ones((2, 4, 4))
    ok = ref + 1e-9
    assert gate(ok, ref, [0, 0]) < 1e-8
    for bad in (np.nan, np.inf):
        C = ok.copy()
        C[1, 2, 3] = bad
        assert gate(C, ref, [0, 0]) == float("inf")
        rep = error_report(C, ref, [0, 0])
        assert rep["gate"] == float("inf") and rep["nonfinite"] == 1


def test_gate_scales_by_row_maximum():
    ref = np.zeros((2, 2, 2))
    ref[0] = 10.0
    ref[1] = 1e-3                    # small block of the same row J
    C = ref.copy()
    C[1] += 1e-9
    assert abs(gate(C, ref, [5, 5]) - 1e-10) < 1e-16
