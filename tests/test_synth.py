"""The input generator's large-instance observation path (band CSR product,
threaded over days) against its element loop, on small shapes including
H != T and links that no route crosses."""
import numpy as np
import pytest

from synth.instances import _BandCSR, _incidence, _lag_ratios, _pattern_csr


@pytest.mark.parametrize("P,L,T,H,K,pattern", [(5, 8, 9, 9, 3, "bernoulli"),
                                                (6, 16, 10, 7, 4, "corridor"),
                                                (4, 9, 6, 11, 3, "bernoulli")])
def test_band_product_matches_element_loop(P, L, T, H, K, pattern):
    rng = np.random.default_rng(5)
    S = _incidence(rng, L, P, 0.15 if pattern == "corridor" else 0.4, pattern)
    row_ptr, col_idx = _pattern_csr(S)
    W = _lag_ratios(rng, K, T, H, col_idx.shape[0])
    Q = rng.uniform(0, 10, (37, T, P))
    band = _BandCSR(P, L, T, H, K, row_ptr, col_idx)
    got = band.product(W, Q).reshape(37, H, L)
    ref = np.zeros((37, H, L))
    rows = np.repeat(np.arange(L), np.diff(row_ptr))
    for l in range(K):
        for t in range(min(T, H - l)):
            for j in range(rows.shape[0]):
                ref[:, t + l, rows[j]] += W[l, t, j] * Q[:, t, col_idx[j]]
    np.testing.assert_allclose(got, ref, rtol=1e-13, atol=1e-12)
    # columns sorted within every row
    for r in range(H * L):
        seg = band.indices[band.indptr[r]:band.indptr[r + 1]]
        assert np.all(np.diff(seg) > 0)
