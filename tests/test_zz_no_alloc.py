"""The non-allocating msCLEAN entry point (GPU required).

imager_minor_cycle_msclean_static runs the minor cycle of
imager_minor_cycle_msclean on a fixed device array instead of the handle's
work area.  Its results must equal the allocating call's bit for bit, on
two calls in a row with the second on a smaller image (the array keeps the
first call's contents), and it must refuse a size beyond its array without
touching the handle's memory.
"""

import numpy as np
import pytest

from helpers import say, to_np, workload

pytestmark = pytest.mark.gpu


def _case(n_pix, scales, niter):
    import torch
    from paper_2507_22128_amd import imager
    d = workload("tiny", n_time=12)
    h = imager.Imager.create(d, n_pix=n_pix, n_partitions=1, weighting="uniform")
    model = torch.zeros((n_pix, n_pix), device="cuda")
    dirty = h.major_cycle(0, model)
    psf = h.psf(0)
    return h, dirty, psf


def _bytes(h):
    h.refresh_info()
    return h.info.device_bytes


def _both(h, dirty, psf, scales, niter):
    bytes0 = _bytes(h)
    got = h.minor_cycle_msclean(0, dirty, psf, scales, niter=niter, static=True)
    bytes1 = _bytes(h)
    ref = h.minor_cycle_msclean(0, dirty, psf, scales, niter=niter)
    return got, ref, bytes0, bytes1


@pytest.mark.parametrize("first,second", [((256, [0, 4, 12], 400), (128, [0, 2], 150))])
def test_static_msclean_equals_allocating_call_twice(first, second):
    for n_pix, scales, niter in (first, second):
        say("case: static msCLEAN, N = %d, S = %s, K = %d" % (n_pix, scales, niter))
        h, dirty, psf = _case(n_pix, scales, niter)
        (d_s, c_s, r_s), (d_r, c_r, r_r), b0, b1 = _both(h, dirty, psf, scales, niter)
        say("  %d components (allocating call: %d)" % (len(c_s), len(c_r)))
        assert len(c_s) > 10
        assert b0 == b1  # the handle's device memory did not grow
        assert np.array_equal(c_s, c_r)
        assert np.array_equal(to_np(d_s), to_np(d_r))
        assert np.array_equal(to_np(r_s), to_np(r_r))
        h.destroy()


def test_static_msclean_refuses_a_size_beyond_its_array():
    from paper_2507_22128_amd import imager
    say("case: static msCLEAN at N = 1024, S = {0, 4, 12} (needs more than the array)")
    h, dirty, psf = _case(1024, [0, 4, 12], 10)
    b0 = _bytes(h)
    with pytest.raises(imager.ImagerError) as e:
        h.minor_cycle_msclean(0, dirty, psf, [0, 4, 12], niter=10, static=True)
    assert e.value.code == imager.EINVAL and "static msCLEAN work area" in str(e.value)
    assert _bytes(h) == b0
    # the handle is still usable afterwards
    _, comps, _ = h.minor_cycle_msclean(0, dirty, psf, [0, 4, 12], niter=10)
    assert len(comps) == 10
    h.destroy()
