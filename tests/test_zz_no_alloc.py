"""The allocation-free error norms (lbm_error_norms_noalloc) against lbm_error_norms: the same
three norms, bitwise, on two calls in a row, the second on a smaller run; every pointer the new
entry point takes is device memory (PyTorch tensors here), and it allocates nothing."""
import numpy as np
import pytest

from paper_2504_20169_amd import lbm
from paper_2504_20169_amd import workloads as wl
from _helpers import say

pytestmark = pytest.mark.gpu


def _run(L, Ly, W, seed):
    mean = (1.0, 0.05, 0.0, 1.0)
    r = lbm.Run(L, Ly, 0.8, *mean)
    r.set_bc(15, "nrbc")
    r.set_pml(15, W, 0.05)
    Nx, Ny = r.grid()
    r.init(*wl.noisy_state(Nx, Ny, seed, *mean).as_tuple())
    r.step(23)
    ref = wl.noisy_state(L, Ly, seed + 100, *mean)
    return r, ref


def test_noalloc_error_norms_equal_the_allocating_entry_point():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("PyTorch in this process sees no HIP device")
    for L, Ly, W, seed in ((90, 70, 6, 3), (30, 20, 4, 5)):   # the second call on a smaller run
        say("case noalloc error norms", L, Ly, W)
        r, ref = _run(L, Ly, W, seed)
        want = r.error_norms(ref.rho, ref.ux, ref.T)
        dev = [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in (ref.rho, ref.ux, ref.T)]
        out = torch.full((3,), float("nan"), dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        r.error_norms_noalloc(dev[0].data_ptr(), dev[1].data_ptr(), dev[2].data_ptr(), out.data_ptr())
        r.synchronize()
        got = out.cpu().numpy()
        say(got, want)
        assert np.array_equal(got, want), (got, want)
        r.close()


def test_noalloc_error_norms_reject_bad_arguments():
    r = lbm.Run(40, 30, 0.8)
    with pytest.raises(lbm.LbmError):          # not initialised
        r.error_norms_noalloc(8, 8, 8, 8)
    r.set_bc(15, "zg")
    r.init(*wl.uniform_state(40, 30).as_tuple())
    with pytest.raises(lbm.LbmError):          # NULL pointer
        r.error_norms_noalloc(0, 8, 8, 8)
    big = lbm.Run(8, 20000, 0.8)               # more bulk rows than the scratch holds
    big.set_bc(15, "periodic")
    big.init(*wl.uniform_state(8, 20000).as_tuple())
    with pytest.raises(lbm.LbmError, match="rows"):
        big.error_norms_noalloc(8, 8, 8, 8)
    big.close()
    r.close()
