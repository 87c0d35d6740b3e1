"""The largest lattices the row form takes, on one GPU: 2^30 nodes with two
FP32 population buffers (210 GB of lattice state) and 2^31 nodes, the
ABI's limit, with one FP16 buffer and the AA pattern (176 GB).  The Couette
start is uniform in x and y, so after a few steps every node of a z layer
must hold the same state, and that state must equal the one of a narrow
lattice with the same walls, bit for bit (each node's update reads only its
own column's values and the same arithmetic runs in both): the velocity
field of every node is compared with the narrow lattice's profile, and the
FP64 totals with the narrow lattice's scaled by the area ratio.  Population
offsets reach 3.3e10 elements here; their 32-bit arithmetic is checked for
every row on the CPU (test_addressing.py)."""
import gc
import sys

import numpy as np
import pytest

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


def column_state(B, shape, storage, one_buffer, steps):
    import torch
    nx, ny, nz = shape
    lat = B.Lattice(nx, ny, nz, 1.0, storage=storage, one_buffer=one_buffer)
    lat.set_shear(0.02, init_profile=True)
    lat.step(steps)
    tot = lat.totals()
    u = lat.velocity()
    # every node of a z layer alike: max == min over x and y, per component
    flat = u.reshape(3, nz, ny * nx)
    uniform = bool(torch.equal(flat.amax(dim=2), flat.amin(dim=2)))
    prof = u[:, :, 0, 0].cpu().numpy()
    del u, flat
    lat.close()
    del lat
    gc.collect()
    torch.cuda.empty_cache()
    return uniform, prof, tot


@pytest.mark.parametrize("shape,storage,one_buffer", [((256, 2048, 2048), "fp32", False),
                                                      ((256, 4096, 2048), "fp16", True)])
def test_largest_lattices(B, shape, storage, one_buffer):
    nx, ny, nz = shape
    say("largest lattice %s %s one buffer %s: %d nodes" % (shape, storage, one_buffer, nx * ny * nz))
    steps = 3  # an odd count: with the AA pattern the state is then the swapped one
    uniform, prof, tot = column_state(B, shape, storage, one_buffer, steps)
    ok_s, prof_s, tot_s = column_state(B, (8, 4, nz), storage, one_buffer, steps)
    area = (nx * ny) / (8 * 4)
    say("  uniform over x and y: %s; profile equal to the narrow lattice's: %s; "
        "mass %.15g vs %.15g" % (uniform, np.array_equal(prof, prof_s), tot[0], tot_s[0] * area))
    assert uniform and ok_s
    assert np.array_equal(prof, prof_s)
    assert np.max(np.abs(prof[0])) > 0.01  # the walls have started the flow
    assert abs(tot[0] - tot_s[0] * area) < 1e-12 * tot[0]
    assert abs(tot[1] - tot_s[1] * area) < 1e-9 * abs(tot[1]) + 1e-6
