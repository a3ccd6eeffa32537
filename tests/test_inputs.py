"""The seeded input generators (shared by tests and benchmark) are deterministic
and fill matrices in the documented column-major draw order."""
import numpy as np

from paper_1303_5837_amd import inputs


def test_gaussian_column_major_draw_order():
    A = inputs.gaussian(7, 3, 123)
    draws = np.random.default_rng(123).standard_normal(21)
    assert A.flags.f_contiguous
    for j in range(3):
        assert np.array_equal(A[:, j], draws[j * 7:(j + 1) * 7])


def test_gaussian_deterministic_and_fp32_rounding():
    a = inputs.gaussian(50, 4, 9)
    b = inputs.gaussian(50, 4, 9)
    assert np.array_equal(a, b)
    c = inputs.gaussian(50, 4, 9, dtype=np.float32)
    assert c.dtype == np.float32 and np.array_equal(c, a.astype(np.float32))


def test_batched_sizes_and_singular_values():
    m, n = inputs.batched_tsqr_sizes(2000)
    assert m.min() >= 256 and m.max() <= 65536 and set(np.unique(n)) <= {8, 16, 32, 64}
    s = inputs.geometric_singular_values(5, 1e4)
    assert s[0] == 1.0 and abs(s[-1] - 1e-4) < 1e-18 and np.all(np.diff(s) < 0)


def test_served_mix_and_arrivals():
    m, n, k = inputs.served_ls_requests(512)
    assert m.min() >= 1024 and m.max() <= 262144 and n.min() >= 16 and n.max() <= 512
    assert np.all(n <= m) and k.min() >= 1e2 and k.max() <= 1e6
    t = inputs.poisson_arrivals(1000.0, 2.0, 11)
    assert np.all(np.diff(t) > 0) and t[-1] < 2.0 and 1800 < len(t) < 2200
    assert np.array_equal(t, inputs.poisson_arrivals(1000.0, 2.0, 11))
