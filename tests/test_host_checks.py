"""Host-side argument checks of the torch binding (no device call is reached on these paths)."""
import numpy as np
import pytest
import torch


def test_short_views_tensor_is_refused():
    """A views tensor must hold n records of sizeof(vf_view) = 72 bytes; one byte short is refused."""
    from paper_2407_14783_amd import capi, sim
    n = 5
    full = torch.zeros(capi.VIEW_DTYPE.itemsize * n, dtype=torch.uint8)
    sim._check_views(full, n)
    with pytest.raises(ValueError):
        sim._check_views(full[:-1], n)
    # the size of the old, wrong record (40 bytes) per view is far too short
    with pytest.raises(ValueError):
        sim._check_views(torch.zeros(40 * n, dtype=torch.uint8), n)


def test_step_and_render_refuse_short_views_before_any_device_call():
    from paper_2407_14783_amd import capi, sim
    from workloads import default_params
    ctx = object.__new__(sim.Context)      # no device context: the check must come first
    ctx.h = None
    n = 4
    short = torch.zeros(capi.VIEW_DTYPE.itemsize * n - 8, dtype=torch.uint8)
    state = torch.zeros((n, 17))
    with pytest.raises(ValueError):
        ctx.step(default_params(), state, torch.zeros((n, 4)), views=short)
    with pytest.raises(ValueError):
        ctx.render(state, short, n=n)
    with pytest.raises(ValueError):
        ctx.collision(state, short, 0.1, n=n)
    with pytest.raises(ValueError):
        ctx.render_backward(state, short, (8, 8), None, None, 0, torch.zeros((n, 17)))


def test_make_views_record_layout():
    """make_views packs 72-byte records with outputs view after view."""
    from paper_2407_14783_amd import capi, sim
    views, npx, offs, mh, mw = sim.make_views(3, [0, 1, 2], [[4, 6], [8, 8], [5, 7]], device="cpu")
    assert views.numel() == 3 * capi.VIEW_DTYPE.itemsize
    rec = np.frombuffer(views.numpy().tobytes(), dtype=capi.VIEW_DTYPE)
    assert list(rec["out_offset"]) == [0, 24, 88] and npx == 24 + 64 + 35 and (mh, mw) == (8, 8)
    assert list(rec["swarm"]) == [0, 0, 0] and np.all(rec["mount_q"][:, 0] == 1.0)
