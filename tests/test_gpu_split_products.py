"""The float matrix-core products of a float32 model (Green's-function Toeplitz products and
the ABACUS deep blocks' channel mixing) in their two arithmetic modes: three-term bf16 splits
on the bf16 matrix cores (the default) and plain float32 matrix cores. Both are compared with
the FP64 oracle on the same inputs. The split mode keeps float32
accuracy: its error bound per product is that of a float32 product (the dropped partial
products are below 2^-24 of each term), so its measured errors must be of the same size as
the plain mode's (within a factor 8 plus 1e-7 absolute, for rounding-order scatter) and
within the float32 parity tolerance 1e-4 (normwise, eps(x) = max|x - x*| / max|x*|)."""
import sys

import pytest
import torch

import dn_inputs as di
import oracle as O
from oracle.model import ModelDesc

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


def eps(x, ref):
    x, ref = torch.as_tensor(x).double().cpu(), torch.as_tensor(ref).double().cpu()
    return (x - ref).abs().max().item() / max(ref.abs().max().item(), 1e-300)


CASES = [
    (di.ModelShape(256, 4, 64, 32, bc="open"), di.HamSpec("lrtfim", "open", alpha=2.0, h=0.5), 3),
    (di.ModelShape(130, 3, 32, 16, bc="periodic"), di.HamSpec("j1j2", "periodic"), 5),
    (di.ModelShape(70, 2, 48, 8, act="tanh", bc="open"), di.HamSpec("lrtfim", "open"), 7),
]


@pytest.mark.parametrize("shape,ham,B", CASES, ids=lambda x: str(x)[:40])
def test_split_products_keep_float32_accuracy(L, shape, ham, B):
    th = torch.tensor(di.draw_params(shape, 61, "stress"))
    sp = di.uniform_spins(B, shape.N, 62)
    M_max = shape.N if ham.kind == "lrtfim" else 2 * shape.N
    ref = O.eloc_plain(ModelDesc.of(shape), ham, th, sp, M_max)
    spd = torch.tensor(sp, device="cuda")
    m = L.Model(shape, "fp32")
    m.set_params(th)
    err = {}
    for mode in ("fp32", "split3"):
        m.set_product_mode(mode)
        for path in ("abacus", "full"):
            lp, lr, el = (t.cpu() for t in m.eloc(ham, spd, M_max, path=path))
            err[mode, path] = (eps(lr, ref["logratio"]), eps(lp, ref["logpsi"]), eps(el, ref["eloc"]))
            _say(f"  {mode} {path}: eps logratio {err[mode, path][0]:.3e} logpsi {err[mode, path][1]:.3e} "
                 f"eloc {err[mode, path][2]:.3e}")
    for path in ("abacus", "full"):
        for e_s, e_f in zip(err["split3", path], err["fp32", path]):
            assert e_s <= 1e-4
            assert e_s <= 8 * e_f + 1e-7, (path, e_s, e_f)
    m.close()


def test_product_mode_argument(L):
    m = L.Model(di.ModelShape(32, 2, 16, 8), "fp32")
    with pytest.raises(L.DysonNetError) as ei:
        L._check(L.lib().dn_set_product_mode(m.handle, 7))
    assert ei.value.status == L.DN_EINVAL
    m.close()
