"""ifl_filter_noalloc against ifl_filter's one-column path (needs MI355X).

The no-allocation entry point runs the one-column kernels with their block
partials and scalars in the library's static device work space. Its results
must be those of ifl_filter with batch = 1 on the same handle (same kernels,
same reduction order: bitwise equal), and within the oracle bars (FP64
<= 1e-11, mixed <= 1e-9). Two calls in a row, the second with a smaller
input (fewer fields and scales, and a smaller mesh whose handle has fewer
logical blocks), check that the shared work space carries nothing over.
"""
import os

import numpy as np
import pytest

import oracle as O
import workloads as W
from oracle.solve import relative_l2

pytestmark = pytest.mark.gpu

TOL = {0: 1e-11, 1: 1e-9}


@pytest.fixture(scope="module")
def ifl():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2404_07398_amd as m

    assert os.path.exists(m.LIB_PATH), "libifl.so must be built before the GPU tests"
    m.lib()
    return m


def _case(level, n_fields, n_scales, seed):
    s = W.icosphere(level, jitter=0.1)
    s = s.with_mask(W.land_mask(s, 0.3))
    phis = np.stack([W.sphere_k3_field(s, seed + f, n_waves=128) for f in range(n_fields)])
    return s, phis, W.log_scales(s.h, n_scales)


@pytest.mark.parametrize("precision", [0, 1])
def test_noalloc_matches_filter_twice(ifl, precision):
    import torch

    dev = torch.device("cuda:0")
    # call 1: level-6 sphere (28k dofs), 2 fields x 4 scales; call 2: level-4
    # sphere, 1 field x 2 scales (fewer blocks, fewer columns)
    for level, nf, ns, seed in ((6, 2, 4, 1000), (4, 1, 2, 1100)):
        s, phis, ks = _case(level, nf, ns, seed)
        print(f"no-alloc case: level {level}, {nf} fields x {ns} scales, precision {precision}", flush=True)
        h = ifl.prepare_mesh(s, 0, 2 if level == 4 else 1, precision=precision, batch=1, device=0)
        L = h.field_length
        f_dev = torch.from_numpy(phis).to(dev)
        ref_out = torch.zeros((nf, ns, L), dtype=torch.float64, device=dev)
        _, ref_stats = h.filter(f_dev, ks, out=ref_out)
        # poison the output so that a missing write shows
        out = torch.full((nf, ns, L), float("nan"), dtype=torch.float64, device=dev)
        stats = h.filter_noalloc(f_dev, ks, out)
        torch.cuda.synchronize()
        a = out.cpu().numpy()
        b = ref_out.cpu().numpy()
        assert np.array_equal(a, b), f"max |diff| {np.nanmax(np.abs(a - b))}"
        for i, (x, y) in enumerate(zip(stats, ref_stats)):
            assert x.status == 0 and y.status == 0
            assert x.iterations == y.iterations, (i, x.iterations, y.iterations)
            assert x.rel_residual == y.rel_residual
        # and the oracle bar of the precision
        op = O.scalar_operator(s, 2 if level == 4 else 1)
        for f in range(nf):
            ref = O.filter_scalar(op, phis[f], ks)
            for j in range(ns):
                err = relative_l2(a[f, j], ref[j])
                assert err <= TOL[precision], (f, j, err)
        h.close()


def test_noalloc_rejects_host_pointers(ifl):
    s, phis, ks = _case(4, 1, 2, 1200)
    h = ifl.prepare_mesh(s, 0, 1, device=0)
    import torch

    out = torch.zeros((1, 2, h.field_length), dtype=torch.float64, device="cuda:0")
    with pytest.raises(ifl.IflError, match="device"):
        h.filter_noalloc(phis, ks, out)
    h.close()
