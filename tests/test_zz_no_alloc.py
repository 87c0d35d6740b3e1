"""The allocation-free variant of the lattice totals (ibm_lattice_totals_noalloc)
against the workspace form (ibm_lattice_totals): two calls in a row on one
GPU, the second on a smaller lattice, each equal to the workspace form bit
for bit (same kernels, same summation order) and to the FP64 sums of the
downloaded populations; a lattice beyond the built-in scratch is refused."""
import sys

import numpy as np
import pytest

from parity_helpers import O
from test_gpu_parity import small_case

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def B():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    from paper_1004_2416_amd import binding
    return binding


def test_totals_noalloc_matches_workspace_form(B):
    import torch
    cvec, _, _ = O.lattice_constants()
    out = torch.full((4,), float("nan"), dtype=torch.float64, device="cuda")
    cases = [(small_case(n=(96, 64, 48), m=3, ca=0.02, perturb=0.02), "fp32", 37),
             (small_case(n=(30, 20, 16), m=2, ca=0.05, perturb=0.01), "fp16", 5)]
    for c, storage, steps in cases:
        lat = c.gpu(storage=storage, graph=True)
        lat.step(steps)
        lat.totals_noalloc(out)
        lat.synchronize()
        got = out.cpu().numpy().copy()
        ref = lat.totals()
        f = lat.populations().cpu().numpy()
        own = np.array([f.sum()] + [np.tensordot(cvec[:, a], f, axes=(0, 0)).sum()
                                    for a in range(3)])
        N = f[0].size
        lat.close()
        say("  %s %s: noalloc %s  workspace %s" % (lat_shape(c), storage, got, ref))
        assert np.array_equal(got, ref)
        assert abs(got[0] - own[0]) < 1e-13 * N
        assert np.max(np.abs(got[1:] - own[1:])) < 1e-13 * N


def lat_shape(c):
    return "%dx%dx%d" % (c.wl.nx, c.wl.ny, c.wl.nz)


def test_totals_noalloc_refuses_lattices_beyond_its_scratch(B):
    import torch
    lat = B.Lattice(512, 256, 257)  # 33.7 M nodes > 8192 partial sums of 4096
    out = torch.zeros(4, dtype=torch.float64, device="cuda")
    with pytest.raises(B.IBMError) as e:
        lat.totals_noalloc(out)
    assert e.value.code == -1 and "workspace" in str(e.value)
    lat.close()
