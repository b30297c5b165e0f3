"""The seeded input generators (shared by the oracle and the HIP path; they
hold none of the method's arithmetic): the threaded R-MAT generator against a
plain sequential restatement of its definition, and the invariants every
generated CSR must satisfy."""
import numpy as np
import pytest

from paper_2212_01473_amd import inputs as I


def _rmat_sequential(scale, edge_factor, a, b, c, seed, chunk):
    """R-MAT by its definition: chunk by chunk and bit by bit from one PCG64
    stream, u < a -> (0,0), < a+b -> (0,1), < a+b+c -> (1,0), else (1,1);
    then self-loops dropped, duplicates removed, symmetrised."""
    n = 1 << scale
    m = n * edge_factor
    rng = np.random.Generator(np.random.PCG64(seed))
    src, dst = [], []
    for start in range(0, m, chunk):
        k = min(chunk, m - start)
        s = np.zeros(k, dtype=np.int64)
        t = np.zeros(k, dtype=np.int64)
        for bit in range(scale - 1, -1, -1):
            u = rng.random(k)
            s |= (u >= a + b).astype(np.int64) << bit
            t |= ((((u >= a) & (u < a + b)) | (u >= a + b + c)).astype(np.int64)) << bit
        src.append(s)
        dst.append(t)
    return I.from_edges(n, np.concatenate(src), np.concatenate(dst))


@pytest.mark.parametrize("scale,ef,chunk,workers", [(8, 16, 1000, 1), (10, 8, 777, 3), (12, 16, 4096, 8),
                                                    (12, 32, 1 << 24, 8)])
def test_rmat_matches_sequential_definition(scale, ef, chunk, workers):
    got = I.rmat(scale, ef, 0.57, 0.19, 0.19, 0.05, 40 + scale, chunk=chunk, workers=workers)
    exp = _rmat_sequential(scale, ef, 0.57, 0.19, 0.19, 40 + scale, chunk)
    assert got.n == exp.n
    assert np.array_equal(got.row_ptr, exp.row_ptr)
    assert np.array_equal(got.col_idx, exp.col_idx)


@pytest.mark.parametrize("make", [lambda: I.rmat(11, 16, 0.57, 0.19, 0.19, 0.05, 3),
                                  lambda: I.erdos_renyi(500, 0.03, 2),
                                  lambda: I.chung_lu_planted(n=3000, wmax=60, n_cliques=5, cmin=10, cmax=20,
                                                             pool=500, seed=4),
                                  lambda: I.planted_partition(400, 8, 0.3, 0.005, 5)])
def test_generated_csr_is_simple_and_symmetric(make):
    g = make()
    rp, ci = g.row_ptr.astype(np.int64), g.col_idx.astype(np.int64)
    assert rp[0] == 0 and rp[-1] == ci.size and np.all(np.diff(rp) >= 0)
    src = np.repeat(np.arange(g.n), np.diff(rp))
    assert np.all(ci < g.n) and np.all(ci != src)
    for v in range(g.n):
        row = ci[rp[v]:rp[v + 1]]
        assert np.all(np.diff(row) > 0)
    fwd = set(zip(src.tolist(), ci.tolist()))
    assert all((u, v) in fwd for v, u in fwd)
