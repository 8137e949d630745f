"""The benchmark's algorithmic byte models (host logic, no GPU)."""
import bench


def test_model_bytes_2d_per_step():
    # float64 step j: 120 N for the four line passes and (3(j+1)+5)*8 N for CGS2
    assert bench.model_bytes_2d(1, 1, 0, 30, False) == 120 + 64
    assert bench.model_bytes_2d(1, 2, 0, 30, False) == (120 + 64) + (120 + 88)
    # a restart resets j
    assert bench.model_bytes_2d(1, 31, 0, 30, False) == bench.model_bytes_2d(1, 30, 0, 30, False) + 184
    # mixed outer step with 16 inner steps: casts 24, inner norm 4, inner steps
    # sum(60 + (2k+3)*4, k = 1..16), update 68, tau 28, matvec 72, CGS2 64
    inner = sum(60 + (2 * k + 3) * 4 for k in range(1, 17))
    assert bench.model_bytes_2d(1, 1, 16, 30, True) == 24 + 4 + inner + 68 + 28 + 72 + 64
    assert bench.model_bytes_2d(1000, 1, 16, 30, True) == 1000 * bench.model_bytes_2d(1, 1, 16, 30, True)


def test_model_bytes_1d_per_step():
    # float64 step j: tau 24 + matvec 32 + CGS2 (32j + 80) + normalisation 16
    assert bench.model_bytes_1d(1, 1, 0, 30, 0, False) == 152
    assert bench.model_bytes_1d(1, 2, 0, 30, 0, False) == 152 + 184
    # float32 preconditioner alone (no inner steps): casts and tau 36 instead of tau 24
    assert bench.model_bytes_1d(1, 1, 0, 30, 0, True) == 32 + 80 + 16 + 36
