"""The loss entry point that allocates nothing (gs_loss_noalloc) against
gs_loss with a caller workspace: two calls in a row through the C ABI, the
second on a smaller image, each bit-identical to gs_loss on the same inputs
(the same kernels run; only where the per-tile partial sums live differs)."""
import ctypes as C

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from gen import images
from paper_2402_17427_amd import _native as N
from paper_2402_17427_amd.raster import stream_handle

pytestmark = pytest.mark.gpu


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else C.c_void_p(0)


def _dev(a):
    return torch.as_tensor(np.ascontiguousarray(a, np.float32)).cuda()


def _both(r, t, lam, ra):
    """(loss, d_image, d_image_l1) from gs_loss with a workspace and from
    gs_loss_noalloc on the same device inputs."""
    Cc, H, W = r.shape
    st = C.c_void_p(stream_handle())
    outs = []
    for noalloc in (False, True):
        loss = torch.full((3,), float("nan"), device="cuda")
        d = torch.full_like(r, float("nan"))
        d1 = torch.full_like(r, float("nan")) if ra is not None else None
        if noalloc:
            N.call("gs_loss_noalloc", _ptr(r), _ptr(ra), _ptr(t), Cc, W, H, C.c_float(lam), _ptr(loss), _ptr(d),
                   _ptr(d1), st)
        else:
            nb = C.c_size_t(0)
            N.call("gs_loss_workspace", Cc, W, H, C.byref(nb))
            ws = torch.empty(max(int(nb.value) // 8, 1), dtype=torch.float64, device="cuda")
            N.call("gs_loss", _ptr(r), _ptr(ra), _ptr(t), Cc, W, H, C.c_float(lam), _ptr(loss), _ptr(d), _ptr(d1),
                   _ptr(ws), C.c_size_t(ws.numel() * 8), st)
        torch.cuda.synchronize()
        outs.append((loss.cpu().numpy(), d.cpu().numpy(), None if d1 is None else d1.cpu().numpy()))
    return outs


def test_loss_noalloc_equals_loss_on_two_calls_in_a_row():
    cases = [((3, 1080, 1920), 0.2, False, 5),    # Eq. 1 at 1080p
             ((3, 61, 97), 0.2, True, 6)]         # then a smaller, ragged Eq. 3 call
    for (Cc, H, W), lam, eq3, seed in cases:
        print(f"\n[case] noalloc {Cc}x{H}x{W} eq3={eq3}", flush=True)
        r, t = images.image_pair(seed, W, H)
        ra = (r * 1.05).astype(np.float32) if eq3 else None
        (l0, d0, e0), (l1, d1, e1) = _both(_dev(r), _dev(t), lam, None if ra is None else _dev(ra))
        assert np.isfinite(l0).all() and np.isfinite(d0).all()
        np.testing.assert_array_equal(l1, l0)
        np.testing.assert_array_equal(d1, d0)
        if eq3:
            np.testing.assert_array_equal(e1, e0)


def test_loss_noalloc_rejects_an_image_beyond_its_scratch():
    big = torch.zeros(1, device="cuda")
    rc = N.lib().gs_loss_noalloc(_ptr(big), None, _ptr(big), 3, 8192, 8192, C.c_float(0.2), _ptr(big), _ptr(big),
                                 None, C.c_void_p(stream_handle()))
    assert rc == N.GS_ERR_CAPACITY, rc
    assert b"partial sums" in N.lib().gs_last_error()
