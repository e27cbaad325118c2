"""The no-allocation Gram entry point (ks_gram_static) against ks_gram through the C ABI:
two calls in a row, the second smaller, and the size limits."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _blocks(torch, n, p, dtype, seed):
    g = torch.Generator().manual_seed(seed)
    A = torch.randn(n, p, generator=g, dtype=torch.float64).to(dtype).cuda()
    B = torch.randn(n, p, generator=g, dtype=torch.float64).to(dtype).cuda()
    return A, B


def _via_system(ks, torch, A, B, grid, prec):
    nx, ny, nz = grid
    p = A.shape[1]
    sysg = ks.KSSystem(ks.make_desc(nx, ny, nz, 0.5, (0, 0, 0), p, precision=prec))
    out = torch.empty(3, p, p, dtype=torch.float64, device="cuda")
    sysg.ks_gram(A, B, out)
    torch.cuda.synchronize()
    sysg.close()
    return out.cpu().numpy()


@pytest.mark.parametrize("dtype_name", ["float64", "float32"])
def test_gram_static_matches_ks_gram_twice(dtype_name):
    import torch
    from paper_1308_2864_amd import ks
    dtype = getattr(torch, dtype_name)
    prec = ks.KS_PREC_FP64 if dtype == torch.float64 else ks.KS_PREC_FP32
    # a large call (more row chunks than the static scratch holds: 128 instead of 512), then
    # a smaller one with a ragged p; the second must not see anything of the first
    for grid, p, seed in (((64, 64, 40), 64, 0), ((17, 13, 11), 23, 1)):
        n = grid[0] * grid[1] * grid[2]
        print(f"# gram_static {dtype_name} n={n} p={p}", flush=True)
        A, B = _blocks(torch, n, p, dtype, seed)
        ref = _via_system(ks, torch, A, B, grid, prec)
        out = torch.full((3, p, p), float("nan"), dtype=torch.float64, device="cuda")
        ks.ks_gram_static(A, B, out)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        # FP64 sums of n products in a different chunk order: rounding only
        scale = np.abs(ref).max()
        assert np.isfinite(got).all()
        assert np.abs(got - ref).max() <= 1e-13 * scale * max(1.0, np.sqrt(n / 4096.0))
        # and against the plain products of the same (rounded) operands
        a = A.double().cpu().numpy()
        b = B.double().cpu().numpy()
        for k, m in enumerate((a.T @ a, a.T @ b, b.T @ b)):
            assert np.abs(got[k] - m).max() <= 1e-12 * np.abs(m).max()


def test_gram_static_rejects_sizes_beyond_its_scratch():
    import ctypes as C
    import torch
    from paper_1308_2864_amd import ks
    A, B = _blocks(torch, 1000, 65, torch.float64, 2)
    out = torch.empty(3, 65, 65, dtype=torch.float64, device="cuda")
    rc = ks.lib.ks_gram_static(C.c_void_p(A.data_ptr()), C.c_void_p(B.data_ptr()), 1000, 65, 65,
                               ks.KS_PREC_FP64, C.c_void_p(out.data_ptr()), None)
    assert rc == ks.KS_E_INVAL
    assert b"64" in ks.lib.ks_last_error(None)
    rc = ks.lib.ks_gram_static(None, C.c_void_p(B.data_ptr()), 1000, 8, 8, ks.KS_PREC_FP64,
                               C.c_void_p(out.data_ptr()), None)
    assert rc == ks.KS_E_INVAL
