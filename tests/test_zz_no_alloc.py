"""lrcc_gemm_noalloc (the GEMM entry point that allocates no device memory)
against lrcc_gemm, through the C ABI: two calls in a row, the second with a
smaller input, both deep enough to be split over K so that the static
split-K scratch is used and reused."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


def _rand(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
def test_gemm_noalloc_matches_gemm_twice(dtype):
    from paper_2503_23144_amd import lrcc
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(7)
    st = torch.cuda.Stream()
    al, be = 0.7 - 0.3j, 0.25 + 0.5j
    # (m, n, k, transa, transb): both shapes split over K; the second is smaller
    for m, n, k, ta, tb in [(960, 150, 9000, False, True), (130, 3, 7000, True, False)]:
        A = _rand(rng, *((k, m) if ta else (m, k)))
        B = _rand(rng, *((n, k) if tb else (k, n)))
        C0 = _rand(rng, m, n)
        Ad = torch.tensor(A, dtype=dtype, device=dev)
        Bd = torch.tensor(B, dtype=dtype, device=dev)
        ref = torch.tensor(C0, dtype=dtype, device=dev)
        got = ref.clone()
        lrcc.gemm(Ad, Bd, ref, transa=ta, transb=tb, alpha=al, beta=be)
        torch.cuda.synchronize()
        print(f"noalloc gemm {dtype} m={m} n={n} k={k}", flush=True)
        with torch.cuda.stream(st):
            lrcc.gemm(Ad, Bd, got, transa=ta, transb=tb, alpha=al, beta=be, stream=st.cuda_stream, noalloc=True)
        st.synchronize()
        r = ref.cpu().numpy().astype(np.complex128)
        g = got.cpu().numpy().astype(np.complex128)
        eps = 1e-15 if dtype == torch.complex128 else 2e-7
        scale = np.sqrt(k) * np.abs(A).max() * np.abs(B).max() + np.abs(C0).max()
        assert np.abs(g - r).max() <= 20 * eps * scale * np.sqrt(k)
        # and against the host product
        host = al * ((A.T if ta else A) @ (B.T if tb else B)) + be * C0
        assert np.abs(g - host).max() <= 20 * eps * scale * np.sqrt(k)


def test_gemm_noalloc_rejects_bad_arguments():
    from paper_2503_23144_amd import lrcc
    dev = torch.device("cuda:0")
    A = torch.zeros((4, 3), dtype=torch.complex128, device=dev)
    B = torch.zeros((3, 6), dtype=torch.complex128, device=dev)
    C = torch.zeros((4, 2), dtype=torch.complex128, device=dev)  # leading dimension 2 < n = 6
    with pytest.raises(lrcc.LrccError, match="leading dimension"):
        lrcc.gemm(A, B, C, noalloc=True)
