"""The entry point that allocates nothing (dn_logpsi_noalloc, through the C ABI) against
dn_logpsi on the same inputs: two calls in a row on one model (the second with fewer
configurations), then a second model of another precision and shape. Both entry points run
the same kernels configuration by configuration, so the bar is float64 rounding (1e-12
relative; the values agree bit for bit in practice)."""
import ctypes
import sys

import pytest
import torch

import dn_inputs as di

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def L():
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    from paper_2603_11189_amd import _lib
    _lib.lib()
    return _lib


def _call(L, m, spins, out):
    st = L.lib().dn_logpsi_noalloc(m.handle, ctypes.c_void_p(spins.data_ptr()), spins.shape[0],
                                   ctypes.c_void_p(out.data_ptr()),
                                   ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    if st != L.DN_OK:
        raise L.DysonNetError(st, L.lib().dn_last_error().decode())
    return out


def _rel(a, b):
    a, b = a.double().cpu(), b.double().cpu()
    return (a - b).abs().max().item() / max(b.abs().max().item(), 1e-300)


CASES = [
    # shape, prec, first B (several scratch chunks), second B
    (di.ModelShape(256, 4, 64, 32, bc="open"), "fp32", 300, 37),
    (di.ModelShape(130, 2, 32, 16, bc="periodic", act="tanh"), "fp64", 90, 5),
    # phi injected into the h stream
    (di.ModelShape(100, 3, 32, 16, bc="periodic", inject_phi=1), "fp32", 120, 9),
]


@pytest.mark.parametrize("shape,prec,B1,B2", CASES, ids=lambda x: str(x)[:40])
def test_noalloc_matches_logpsi(L, shape, prec, B1, B2):
    m = L.Model(shape, prec)
    m.set_params(torch.tensor(di.draw_params(shape, 71, "stress")))
    for B, seed in ((B1, 5), (B2, 6)):
        sp = torch.tensor(di.uniform_spins(B, shape.N, seed), device="cuda")
        ref = m.logpsi(sp)
        out = torch.full((B,), float("nan"), dtype=torch.float64, device="cuda")
        _call(L, m, sp, out)
        torch.cuda.synchronize()
        e = _rel(out, ref)
        _say(f"noalloc {shape.N} L{shape.L} d{shape.d} {prec} B={B}: rel err vs dn_logpsi {e:.3e}, "
             f"bit-equal {torch.equal(out, ref)}")
        assert torch.isfinite(out).all()
        assert e <= 1e-12
    m.close()


def test_noalloc_argument_errors(L):
    shape = di.ModelShape(16, 1, 8, 4, act="tanh")
    m = L.Model(shape, "fp64")
    sp = torch.tensor(di.uniform_spins(2, 16, 1), device="cuda")
    out = torch.empty(2, dtype=torch.float64, device="cuda")
    with pytest.raises(L.DysonNetError) as ei:
        _call(L, m, sp, out)  # no parameters yet
    assert ei.value.status == L.DN_ESTATE
    m.set_params(torch.tensor(di.draw_params(shape, 1, "baseline")))
    st = L.lib().dn_logpsi_noalloc(m.handle, ctypes.c_void_p(sp.data_ptr()), -1, ctypes.c_void_p(out.data_ptr()),
                                   None)
    assert st == L.DN_EINVAL
    st = L.lib().dn_logpsi_noalloc(m.handle, None, 2, ctypes.c_void_p(out.data_ptr()), None)
    assert st == L.DN_EINVAL
    m.close()
