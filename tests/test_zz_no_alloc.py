"""The entry point that allocates nothing, gicp_covariances_noalloc, through
the C ABI against gicp_covariances (the same kernels on a library-owned
workspace): bitwise-equal covariances on calls in a row, the first at the
maximum size and the later ones smaller; an input above the fixed workspace
is refused with its own status."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[case]", *a, flush=True)


def test_noalloc_equals_covariances():
    import torch

    import paper_2403_12550_amd as g
    from paper_2403_12550_amd import _abi
    torch.cuda.set_device(0)
    ctx = g.Context(0)
    nmax = _abi.NOALLOC_MAX_POINTS
    big = g.to_soa(synth.c1_problem(n=nmax, src_seed=7).src)
    small = g.to_soa(synth.c1_problem(n=5000, src_seed=8).src)
    cases = [(big, 0.05, g.REG_PLANE), (small, 0.1, g.REG_PLANE), (small, 0.0, g.REG_ELLIPSE),
             (small[:, :777].contiguous(), 0.0, g.REG_NONE)]
    for pts, cell, mode in cases:
        n = pts.shape[1]
        _say("noalloc", n, cell, mode)
        h = cell if cell > 0 else ctx.estimate_cell(pts, 20)
        a = ctx.covariances_noalloc(pts, 20, cell=cell, reg_mode=mode)
        b = ctx.covariances(pts, 20, cell=h, reg_mode=mode)
        torch.cuda.synchronize()
        assert torch.equal(a.view(torch.int32), b.view(torch.int32)), (n, cell, mode)
    # the first case again after smaller ones: the shared array's old contents do not leak in
    a = ctx.covariances_noalloc(big, 20, cell=0.05, reg_mode=g.REG_PLANE)
    b = ctx.covariances(big, 20, cell=0.05, reg_mode=g.REG_PLANE)
    assert torch.equal(a.view(torch.int32), b.view(torch.int32))
    over = g.to_soa(synth.c1_problem(n=nmax + 1, src_seed=9).src)
    with pytest.raises(g.GicpError) as e:
        ctx.covariances_noalloc(over, 20, cell=0.05)
    assert e.value.status == _abi.GICP_E_TOO_LARGE
    ctx.close()
