"""The allocation-free entry point dbfft_apply_noalloc against dbfft_apply.

Both are called through the C ABI on the same seeded inputs; the
allocation-free one twice in a row on the same stream, the second call on a
smaller grid (so it must not depend on what the first left in its static
workspace), and the results are compared with a context's dbfft_apply to
the FP64 operator bar (1e-12 relative, max-norm; the two differ only in how
the twiddle tables were rounded).  A grid whose workspace exceeds the static
array is rejected before any GPU work, and an out-of-range phase id gives a
NaN output.
"""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def _noalloc(n, material, field, params, u, f, stream):
    from paper_1905_12725_amd import _native as nat
    nn = (ctypes.c_int64 * 3)(*n)
    pp = (ctypes.c_double * len(params))(*params)
    return nat.lib().dbfft_apply_noalloc(nn, material, _ptr(field), pp, len(params), _ptr(u), _ptr(f),
                                         ctypes.c_void_p(stream))


def _reference(n, kind, field, params, u):
    from paper_1905_12725_amd.api import Cell
    with Cell(n, kind, field, params) as cell:
        return cell.apply(u).cpu().numpy()


@pytest.mark.parametrize("material", ["iso_phase", "iso_field"])
def test_noalloc_matches_apply_two_calls(gpu, material):
    import torch
    from paper_1905_12725_amd import _native as nat
    stream = torch.cuda.current_stream().cuda_stream
    rng = np.random.default_rng(700)
    cases = [(64, 48, 80), (20, 18, 30)]  # second call: smaller grid
    outs, refs = [], []
    for n in cases:
        print(f"case noalloc {material} n={n}", flush=True)
        if material == "iso_phase":
            field = torch.from_numpy((rng.random(n) < 0.35).astype(np.uint8)).cuda()
            params = [1.0, 0.3, 7.0, 0.25]
            mat = nat.MAT_ISO_PHASE
        else:
            field = torch.from_numpy(np.exp(rng.standard_normal(n))).cuda()
            params = [0.3]
            mat = nat.MAT_ISO_FIELD
        u = torch.from_numpy(rng.standard_normal((3,) + n)).cuda()
        f = torch.full_like(u, float("nan"))
        nat.check(_noalloc(n, mat, field, params, u, f, stream))
        outs.append((f, field, params, u, n))
    torch.cuda.synchronize()
    for f, field, params, u, n in outs:
        refs.append(_reference(n, material, field, params, u))
    for (f, _, _, _, n), ref in zip(outs, refs):
        got = f.cpu().numpy()
        assert np.all(np.isfinite(got)), n
        assert rel(got, ref) < 1e-12, (n, rel(got, ref))


def test_noalloc_rejects_grids_above_its_workspace(gpu):
    import torch
    from paper_1905_12725_amd import _native as nat
    n = (96, 96, 96)
    field = torch.zeros(n, dtype=torch.uint8, device="cuda")
    u = torch.zeros((3,) + n, dtype=torch.float64, device="cuda")
    f = torch.zeros_like(u)
    st = _noalloc(n, nat.MAT_ISO_PHASE, field, [1.0, 0.3], u, f, torch.cuda.current_stream().cuda_stream)
    assert st == nat.DBFFT_EUNSUPPORTED
    assert "scratch" in nat.lib().dbfft_last_error().decode()


def test_noalloc_flags_out_of_range_phase(gpu):
    import torch
    from paper_1905_12725_amd import _native as nat
    n = (8, 8, 8)
    rng = np.random.default_rng(701)
    ph = (rng.random(n) < 0.5).astype(np.uint8)
    ph[3, 4, 5] = 2  # two phases given
    field = torch.from_numpy(ph).cuda()
    u = torch.from_numpy(rng.standard_normal((3,) + n)).cuda()
    f = torch.zeros_like(u)
    stream = torch.cuda.current_stream().cuda_stream
    nat.check(_noalloc(n, nat.MAT_ISO_PHASE, field, [1.0, 0.3, 5.0, 0.3], u, f, stream))
    torch.cuda.synchronize()
    assert torch.isnan(f).all()
    # a valid call afterwards is not affected by the flag the previous one left
    field.clamp_(max=1)
    nat.check(_noalloc(n, nat.MAT_ISO_PHASE, field, [1.0, 0.3, 5.0, 0.3], u, f, stream))
    torch.cuda.synchronize()
    ref = _reference(n, "iso_phase", field, [1.0, 0.3, 5.0, 0.3], u)
    assert rel(f.cpu().numpy(), ref) < 1e-12
