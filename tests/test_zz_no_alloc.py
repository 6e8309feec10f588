"""The allocation-free Haar entry point against the allocating one.

syk_haar_state_noalloc keeps its norm partial sums in the library's fixed device scratch
instead of a workspace; both entry points run the same kernels in the same order, so the
states must agree bit for bit.  Two calls in a row, the second on a smaller block, check
that the scratch left by the first call does not leak into the second.  Both calls go
through the C ABI (the binding only marshals the arguments)."""
import pytest
import torch

import paper_2311_00639_amd as syk

pytestmark = pytest.mark.gpu


def _pair(N, dtype):
    n = 1 << (N // 2 - 1)
    return (torch.empty(n, dtype=dtype, device="cuda"), torch.empty(n, dtype=dtype, device="cuda"))


@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
def test_noalloc_haar_equals_allocating_entry_point(dtype):
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    # first call on a large block (2048 partial sums), then on a smaller one (fewer partials)
    for N, seed, v in ((46, 4242, 3), (30, 77, 0)):
        ref_u, ref_d = _pair(N, dtype)
        out_u, out_d = _pair(N, dtype)
        out_u.fill_(float("nan"))
        out_d.fill_(float("nan"))
        print(f"[no-alloc] N={N} seed={seed} v={v} dtype={dtype}", flush=True)
        syk.haar_state(N, seed, v, ref_u, ref_d, stream=stream)
        syk.haar_state_noalloc(N, seed, v, out_u, out_d, stream=stream)
        torch.cuda.synchronize()
        assert torch.equal(out_u, ref_u) and torch.equal(out_d, ref_d), N
        norm2 = float((out_u.abs() ** 2).sum(dtype=torch.float64) + (out_d.abs() ** 2).sum(dtype=torch.float64))
        tol = 1e-12 if dtype == torch.complex128 else 1e-5
        assert abs(norm2 - 1.0) < tol, norm2


def test_noalloc_haar_rejects_bad_arguments():
    torch.cuda.set_device(0)
    u, d = _pair(20, torch.complex64)
    with pytest.raises(syk.SykError):
        syk._lib._check(syk._lib._lib.syk_haar_state_noalloc(20, 1, 0, syk.C64, None, d.data_ptr(), None))
    with pytest.raises(syk.SykError):
        syk._lib._check(syk._lib._lib.syk_haar_state_noalloc(21, 1, 0, syk.C64, u.data_ptr(), d.data_ptr(), None))
