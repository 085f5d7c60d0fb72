"""The allocation-free variant of the right-hand-side preparation
(cfd_rhs_prepare_noalloc, through the C ABI) gives the bits of
cfd_rhs_prepare, on two calls in a row, the second with a smaller input."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def test_noalloc_rhs_prepare_matches_the_allocating_call():
    import paper_2504_03697_amd as m
    m.load()
    # larger first, then smaller: the second call reuses the fixed array,
    # which still holds the first call's partial sums
    for dims, pin in (((96, 80, 72), 0), ((17, 13, 11), 100)):
        A = m.assemble(dims, pin)
        b = synth.uniform_rhs(dims, 7) + 0.25
        ref = m.rhs_prepare(A, torch.from_numpy(b).cuda())
        got = m.rhs_prepare_noalloc(A, torch.from_numpy(b).cuda())
        torch.cuda.synchronize()
        ref, got = ref.cpu().numpy(), got.cpu().numpy()
        assert np.array_equal(got, ref), dims
        assert got[pin] == 0.0


def test_noalloc_rejects_null_arguments():
    import paper_2504_03697_amd as m
    from paper_2504_03697_amd import _lib
    lib = m.load()
    A = m.assemble((4, 4, 4), 0)
    assert lib.cfd_rhs_prepare_noalloc(None, None, None) == _lib.CFD_EINVAL
    assert lib.cfd_rhs_prepare_noalloc(A.handle, None, None) == _lib.CFD_EINVAL
