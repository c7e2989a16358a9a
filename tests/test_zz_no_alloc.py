"""The no-allocation propagator entry point (pd_steps_dev_noalloc): the same
results as pd_steps_dev, called twice in a row (the second call smaller, so
stale workspace contents from the first would show), for both steppers, and
a clear error for a batch beyond the static workspace."""
import numpy as np
import pytest

from oracle import spectral as osp
from synthetic import initial_field

pytestmark = pytest.mark.gpu


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _rand(N, batch, seed):
    rng = np.random.default_rng(seed)
    b = rng.standard_normal((batch, 3, N, N)) + 1j * rng.standard_normal((batch, 3, N, N))
    return b * osp.box_mask(N)


@pytest.mark.parametrize("scheme", ["sbdf2", "rk443"])
@pytest.mark.parametrize("N,big,small", [(64, 12, 5), (128, 20, 3), (512, 2, 1)])
def test_noalloc_equals_allocating_entry_point(lib, scheme, N, big, small):
    import torch
    print(f"noalloc N={N} scheme={scheme} batches {big},{small}", flush=True)
    if scheme == "rk443" and N == 512:
        big = 1
    with lib.Context(0) as ctx:
        ctx.set_problem("gp", 80.0, 0.57, N)
        ctx.set_scheme(scheme, "sbdf2")
        ctx.set_path(0)
        for batch, seed in ((big, 1), (small, 2)):
            x = _dev(_rand(N, batch, N + seed))
            t0 = np.linspace(0.3, 4.1, batch)
            ref = ctx.steps(t0, 2e-3, 3, x)
            out = torch.empty_like(x)
            got = ctx.steps_noalloc(t0, 2e-3, 3, x, out)
            torch.cuda.synchronize()
            assert torch.equal(got, ref), (batch, float((got - ref).abs().max()))


def test_noalloc_rejects_a_batch_beyond_the_workspace(lib):
    import torch
    with lib.Context(0) as ctx:
        ctx.set_problem("gp", 80.0, 0.57, 512)
        x = torch.zeros((3, 3, 512, 512), dtype=torch.complex128, device="cuda")
        with pytest.raises(lib.PitdynError) as e:
            ctx.steps_noalloc(np.zeros(3), 1e-3, 1, x, torch.empty_like(x))
        assert e.value.status == lib.EINVAL and "static workspace" in str(e.value)
        # a field outside the 2/3 box is rejected as by pd_steps_dev
        bad = torch.zeros((1, 3, 64, 64), dtype=torch.complex128, device="cuda")
        bad[0, 0, 32, 0] = 1.0
        ctx.set_problem("gp", 80.0, 0.57, 64)
        with pytest.raises(lib.PitdynError) as e:
            ctx.steps_noalloc([0.0], 1e-3, 1, bad, torch.empty_like(bad))
        assert e.value.status == lib.EINVAL
        # the call after the error still works
        y = _dev(initial_field(64, 0.57, 3)[None])
        assert torch.equal(ctx.steps_noalloc([0.0], 1e-3, 2, y, torch.empty_like(y)),
                           ctx.steps([0.0], 1e-3, 2, y))
