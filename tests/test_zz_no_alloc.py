"""mps_norm_noalloc (the entry point that allocates nothing) against mps_norm,
through the C ABI, on two calls in a row (the second on a smaller state),
plus its size limit and that it draws nothing from the device allocator."""
import ctypes as C

import numpy as np
import pytest

from workloads import circuits

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    from paper_2303_11409_amd import MPS, TorchDevice, binding
    return MPS, TorchDevice, binding


def abi_norms(binding, m):
    lib = binding.lib()
    a, b = C.c_double(0.0), C.c_double(0.0)
    assert lib.mps_norm(m._h, C.byref(a)) == 0
    assert lib.mps_norm_noalloc(m._h, C.byref(b)) == 0, lib.mps_last_error().decode()
    return a.value, b.value


def test_noalloc_norm_equals_mps_norm(env):
    MPS, TorchDevice, binding = env

    class Counting(TorchDevice):
        def __init__(self):
            super().__init__()
            self.calls = 0
            inner = self._alloc_cb

            def alloc(nbytes, ctx):
                self.calls += 1
                return inner(nbytes, ctx)

            self._alloc_cb = binding.ALLOC_FN(alloc)

    dev = Counting()
    # a truncated 32-mode circuit (bond dimension up to 256 after 10 layers) ...
    cfg = circuits.config_plain_gpu()
    big = MPS(cfg["occupation"], 4, chi_max=512, cutoff=1e-12, device=dev)
    for lay in cfg["layers"][:10]:
        big.apply_layer([g.site for g in lay], [g.u for g in lay])
    # ... then a smaller state: the 8-mode Clements circuit
    ecfg = circuits.config_small_exact()
    small = MPS(ecfg["occupation"], 5, device=dev)
    for g in ecfg["gates"]:
        small.apply_gate(g.site, g.u)
    assert max(small.bond_dims()) < max(big.bond_dims())
    for m in (big, small):
        ref, got = abi_norms(binding, m)
        assert abs(got - ref) <= 1e-10 * abs(ref), (got, ref)
        before = dev.calls
        assert m.norm2_noalloc() == got          # same result on a repeated call
        assert dev.calls == before               # no device allocation
    assert abs(small.norm2_noalloc() - 1.0) <= 1e-12
    big.close()
    small.close()


def test_noalloc_norm_refuses_a_state_beyond_its_scratch(env):
    MPS, TorchDevice, binding = env
    from paper_2303_11409_amd import MPSError
    ch, gam, lam = circuits.synthetic_state(20, 10, 4, 1024, seed=5)
    m = MPS.from_vidal(4, 10, ch, gam, lam)
    assert max(m.bond_dims()) == 1024
    with pytest.raises(MPSError) as e:
        m.norm2_noalloc()
    assert e.value.status == -1 and "scratch" in str(e.value)
    # the handle is untouched and the allocating path still works
    assert np.isfinite(m.norm2())
    m.close()
