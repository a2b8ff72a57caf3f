"""The Gaussian test matrix of the randomized scheme (Section 4.3) on the GPU
(hmat_gaussian_panel), the generator every sketch uses.

Pinned against the oracle's Philox4x32-10 + Box-Muller (oracle/philox.py, itself pinned
by the published known-answer vectors): the same counters and key give the same 53-bit
uniforms, so the two differ only in the last bits of log and cos (1e-14 absolute).
Moments of a 4-million-entry panel are those of N(0, 1) within five standard errors
(mean, variance, fourth moment), columns are uncorrelated, and a different seed gives a
different panel. Sizes 0 and invalid arguments are checked."""

import numpy as np
import pytest

from oracle import philox

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def H():
    from paper_1805_08998_amd import hmat
    hmat.lib()
    return hmat


def panel(H, n, ncol, seed):
    import torch
    out = torch.empty((ncol, n), dtype=torch.float64, device="cuda")  # column-major n x ncol
    H.hmat_gaussian_panel(n, ncol, seed, out.data_ptr())
    return out.cpu().numpy().T


def test_matches_oracle_generator(H):
    for n, ncol, seed in ((1000, 5, 0x5EED), (3001, 3, 123456789012345), (64, 17, 0)):
        G = panel(H, n, ncol, seed)
        ref = philox.omega(np.arange(n), np.arange(ncol), seed)
        err = np.abs(G - ref).max()
        print(f"n {n} ncol {ncol} seed {seed}: max |GPU - oracle| = {err:.2e}", flush=True)
        assert G.shape == (n, ncol) and err <= 1e-13


def test_rows_beyond_2_32_use_the_high_counter_word(H):
    """Row i enters the counter as (i mod 2^32, j, i div 2^32): one column of 2^32 + 16
    rows (34 GB on the device), its rows on both sides of 2^32 against the oracle."""
    import torch
    n = (1 << 32) + 16
    out = torch.empty(n, dtype=torch.float64, device="cuda")
    H.hmat_gaussian_panel(n, 1, 99, out.data_ptr())
    rows = np.array([0, (1 << 32) - 2, (1 << 32) - 1, 1 << 32, (1 << 32) + 15])
    got = out[torch.from_numpy(rows).cuda()].cpu().numpy()
    del out
    torch.cuda.empty_cache()
    ref = philox.omega(rows, np.arange(1), 99)[:, 0]
    assert np.abs(got - ref).max() <= 1e-13
    # rows 2^32 + r and r share the low counter word and differ in the high one
    assert got[3] != got[0]


def test_moments(H):
    n, ncol = 1 << 20, 4
    G = panel(H, n, ncol, 2024)
    x = G.ravel()
    N = x.size
    mean, var = x.mean(), x.var()
    m4 = np.mean((x - mean) ** 4)
    print(f"N {N}: mean {mean:.2e}, variance {var:.5f}, fourth moment {m4:.4f}", flush=True)
    assert abs(mean) < 5 / np.sqrt(N)
    assert abs(var - 1) < 5 * np.sqrt(2 / N)
    assert abs(m4 - 3) < 5 * np.sqrt(96 / N)
    c = np.corrcoef(G.T)
    assert np.abs(c - np.eye(ncol)).max() < 5 / np.sqrt(n)
    G2 = panel(H, 4096, 1, 2025)
    assert not np.allclose(G2[:, 0], G[:4096, 0])


def test_arguments(H):
    import ctypes
    import torch
    out = torch.empty(8, dtype=torch.float64, device="cuda")
    H.hmat_gaussian_panel(0, 3, 1, out.data_ptr())  # nothing to write
    H.hmat_gaussian_panel(8, 0, 1, out.data_ptr())
    L = H.lib()
    assert L.hmat_gaussian_panel(8, 1, 1, None, None) == H.HMAT_ERR_ARG
    assert L.hmat_gaussian_panel(-1, 1, 1, ctypes.c_void_p(out.data_ptr()), None) == H.HMAT_ERR_ARG
    assert L.hmat_gaussian_panel(8, -2, 1, ctypes.c_void_p(out.data_ptr()), None) == H.HMAT_ERR_ARG
