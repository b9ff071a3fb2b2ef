"""hsym_kernel_gram_noalloc (partials in the library's static device scratch)
against hsym_kernel_gram (partials allocated per call), through the C ABI:
bitwise equal results (the same kernels and the same fixed-order reduction),
on two calls in a row, the second smaller than the first, so that what the
first call left in the scratch cannot leak into the second; and the
size checks."""
import numpy as np
import pytest

import hsymgen

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1609_01689_amd as hs  # noqa: E402


def blocks(seed, n, m, k):
    return [torch.from_numpy(hsymgen.gauss_block(seed + i, n, m)).to("cuda:0") for i in range(k)]


def test_gram_noalloc_matches_allocating_gram():
    stream = torch.cuda.current_stream()
    for n, m, na, nb in [(1_000_003, 16, 3, 6), (70_001, 8, 2, 3)]:
        A = blocks(11, n, m, na)
        B = blocks(41, n, m, nb)
        G0 = torch.full((na * m, nb * m), np.nan, dtype=torch.float64, device="cuda:0")
        G1 = torch.full_like(G0, np.nan)
        hs.hsym_kernel_gram(A, B, G0)
        hs.hsym_kernel_gram_noalloc(A, B, G1, stream=stream)
        torch.cuda.synchronize()
        g0, g1 = G0.cpu().numpy(), G1.cpu().numpy()
        ref = np.concatenate([a.cpu().numpy() for a in A], 1).T @ np.concatenate([b.cpu().numpy() for b in B], 1)
        print("n=%d m=%d %dx%d: max |noalloc - alloc| = %.3g, max rel vs host = %.2e" %
              (n, m, na, nb, np.max(np.abs(g1 - g0)), np.max(np.abs(g1 - ref)) / np.max(np.abs(ref))), flush=True)
        assert np.array_equal(g0, g1)
        assert np.max(np.abs(g1 - ref)) <= 1e-12 * np.max(np.abs(ref)) * np.sqrt(n)


def test_gram_noalloc_rejects_bad_shapes():
    A = blocks(1, 1000, 16, 4)
    G = torch.empty((64, 64), dtype=torch.float64, device="cuda:0")
    with pytest.raises(hs.HsymError):
        hs.hsym_kernel_gram_noalloc(A, A, G)          # na = 4 > 3
    B = blocks(2, 1000, 16, 7)
    with pytest.raises(hs.HsymError):
        hs.hsym_kernel_gram_noalloc(A[:1], B, G)      # nb = 7 > 6
