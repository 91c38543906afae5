"""The seeded input generators: documented fingerprints of each workload
recipe (numpy PCG64 draws of the full matrix, upper triangle kept, cast),
zero lower triangles and padding, inclusive integer ranges.  The expected
numbers were computed independently from the written recipes."""
import numpy as np

from paper_2310_19373_amd import inputs


def test_n20_float_fingerprint():
    q = inputs.single_n20_f32()
    assert q.dtype == np.float32 and q.shape == (20, 20)
    assert np.allclose(q[0, :4], [0.12573022, -0.13210486, 0.64042264, 0.10490011], rtol=0, atol=1e-8)
    assert abs(float(q[19, 19]) - 0.4439914) < 1e-7
    assert abs(float(np.abs(q.astype(np.float64)).sum()) - 177.150442) < 1e-5
    assert np.all(np.tril(q, -1) == 0)


def test_n32_int_fingerprint_and_inclusive_range():
    q = inputs.single_n32_i32()
    assert q.dtype == np.int32 and q.shape == (32, 32)
    assert int(np.abs(q.astype(np.int64)).sum()) == 26352
    assert q.min() >= -100 and q.max() <= 100
    assert np.all(np.tril(q, -1) == 0)
    big = inputs.random_i32(200, 5)  # 20100 draws: both ends of [-100, 100] occur
    assert int(big.min()) == -100 and int(big.max()) == 100


def test_batched_4096_fingerprint():
    q, ns = inputs.batched_4096()
    assert q.shape == (4096, 28, 28) and q.dtype == np.float32 and ns.dtype == np.int32
    assert int(ns.min()) == 12 and int(ns.max()) == 28
    assert int(np.sum(np.ldexp(1.0, ns))) == 128678391808
    assert int((ns == 28).sum()) == 248
    for b in range(0, 4096, 97):
        n = int(ns[b])
        assert np.all(q[b, n:, :] == 0) and np.all(q[b, :, n:] == 0)
        assert np.all(np.tril(q[b], -1) == 0)


def test_logz_pairs_layout():
    q, beta = inputs.logz_256x24()
    assert q.shape == (768, 24, 24) and beta.shape == (768,)
    assert beta[:6].tolist() == [0.5, 1.0, 4.0, 0.5, 1.0, 4.0]
    assert np.array_equal(q[0], q[1]) and np.array_equal(q[0], q[2]) and not np.array_equal(q[0], q[3])
    sd = float(np.std(q[:, np.triu_indices(24)[0], np.triu_indices(24)[1]]))
    assert abs(sd - 1 / np.sqrt(24)) < 0.01  # "N(0, 1/n)": variance 1/n
    assert np.all(np.tril(q, -1) == 0)
