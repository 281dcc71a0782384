"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Error measures (normwise, over batch and elements): eps(x) = max|x - x*| / max|x*|.
Tolerances:
  * float64 mode: 1e-10 (the oracle's own ABACUS == plain agreement is ~1e-15).
  * float32 mode: fields carry unit roundoff u = 6e-8; a channel contraction of d terms and
    a mixer sum of N terms each add ~sqrt(n) u relative error per block, so with L <= 4
    blocks the network output Omega is good to ~1e-5 relative and ABACUS's dOmega, which is
    formed directly, to the same relative level: log-ratios and E_loc are checked to 1e-4.
    The plain path subtracts two full evaluations, so its log-ratio error scales with
    |Omega| |dOmega| rather than with the ratio: it is checked to 1e-4 relative to
    max(|ratio|, |Omega|^2).
  * A pair exchange (J1-J2) changes two spins in opposite directions; its ratio is the
    near-cancelling sum of two single-flip changes, so its rounding error scales with the
    single-flip ratios of the same sample, and pair ratios are checked relative to the larger
    of the pair and single-flip magnitudes.
Integer outputs (sites, n_conn) are compared bit for bit.
"""
import math
import sys

import numpy as np
import pytest
import torch

import dn_inputs as di
import oracle as O
from oracle.model import ModelDesc, forward, s4_taps, unpack

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


def _model(L, shape, seed, scale, prec):
    th = torch.tensor(di.draw_params(shape, seed, scale))
    m = L.Model(shape, prec)
    m.set_params(th)
    return m, th


TAP_SHAPES = [
    di.ModelShape(16, 1, 8, 4, act="tanh", bc="open"),
    di.ModelShape(64, 2, 32, 16, bc="open"),
    di.ModelShape(37, 2, 5, 7, bc="periodic"),
    di.ModelShape(128, 4, 64, 32, bc="periodic"),
    di.ModelShape(256, 4, 64, 32, bc="open"),
]


@pytest.mark.parametrize("shape", TAP_SHAPES, ids=lambda s: f"N{s.N}L{s.L}d{s.d}s{s.s}{s.bc}")
@pytest.mark.parametrize("scale", ["baseline", "stress"])
def test_taps_match_oracle(L, shape, scale):
    _say("taps", shape, scale)
    m, th = _model(L, shape, 77, scale, "fp32")
    taps = m.get_taps().cpu()
    desc = ModelDesc.of(shape)
    prm = unpack(desc, th)
    ref = torch.stack([s4_taps(desc, p4) for p4 in prm["s4"]])
    e = eps(taps, ref)
    _say("  eps", e)
    assert e <= 1e-12


HAMS = [
    (di.HamSpec("lrtfim", "open", J=1.0, alpha=3.0, h=1.0), 20),
    (di.HamSpec("lrtfim", "periodic", J=-1.2, alpha=2.5, h=0.4, paper_form=1), 21),
    (di.HamSpec("j1j2", "periodic", J1=1.0, J2=0.5), 20),
    (di.HamSpec("j1j2", "open", J1=0.7, J2=0.3), 17),
]


@pytest.mark.parametrize("ham,N", HAMS, ids=lambda x: str(x)[:40])
def test_connected_match_oracle(L, ham, N):
    _say("connected", ham, N)
    sp = di.uniform_spins(24, N, 5)
    M_max = N if ham.kind == "lrtfim" else 2 * N
    s, he, nc, hd = L.connected(ham, torch.tensor(sp, device="cuda"), M_max)
    rs, rhe, rnc, rhd = O.connected(ham, sp, M_max)
    assert torch.equal(nc.cpu().long(), rnc)
    assert torch.equal(s.cpu().long(), rs)
    assert torch.allclose(he.cpu(), rhe, rtol=0, atol=0)
    assert eps(hd, rhd) <= 1e-13


FWD_CASES = [
    (di.ModelShape(16, 1, 8, 4, act="tanh", bc="open"), "fp64"),
    (di.ModelShape(24, 3, 8, 4, act="silu", bc="periodic"), "fp64"),
    (di.ModelShape(20, 2, 5, 3, act="identity", bc="open"), "fp64"),
    (di.ModelShape(18, 2, 6, 3, act="tanh", bc="open", inject_phi=1), "fp64"),
    (di.ModelShape(64, 2, 32, 16, bc="open"), "fp32"),
    (di.ModelShape(100, 3, 20, 8, bc="periodic"), "fp32"),
]


@pytest.mark.parametrize("shape,prec", FWD_CASES, ids=lambda x: str(x)[:48])
@pytest.mark.parametrize("scale", ["baseline", "stress"])
def test_logpsi_match_oracle(L, shape, prec, scale):
    _say("logpsi", shape, prec, scale)
    m, th = _model(L, shape, 13, scale, prec)
    sp = di.uniform_spins(70, shape.N, 9)
    lp = m.logpsi(torch.tensor(sp, device="cuda")).cpu()
    fw = forward(ModelDesc.of(shape), th, sp)
    e = eps(lp, fw["logpsi"])
    _say("  eps_logpsi", e)
    assert e <= (1e-10 if prec == "fp64" else 1e-4)


LR_CASES = [
    # shape, ham, prec, B
    (di.ModelShape(16, 1, 8, 4, act="tanh", bc="open"), di.HamSpec("lrtfim", "open"), "fp64", 6),
    (di.ModelShape(20, 2, 8, 4, act="silu", bc="open"), di.HamSpec("lrtfim", "open", alpha=2.0, h=0.5), "fp64", 4),
    (di.ModelShape(22, 3, 6, 3, act="tanh", bc="open"), di.HamSpec("j1j2", "open"), "fp64", 3),
    (di.ModelShape(20, 4, 8, 4, act="silu", bc="periodic"), di.HamSpec("j1j2", "periodic"), "fp64", 3),
    (di.ModelShape(19, 2, 4, 2, act="identity", bc="periodic"), di.HamSpec("lrtfim", "periodic", paper_form=1), "fp64", 3),
    (di.ModelShape(64, 2, 32, 16, bc="open"), di.HamSpec("lrtfim", "open"), "fp32", 4),
    (di.ModelShape(70, 3, 20, 8, bc="periodic"), di.HamSpec("j1j2", "periodic"), "fp32", 3),
    # two blocks with pair exchanges (clusters two sites wide), 64 channels, across the seam
    (di.ModelShape(40, 2, 64, 32, bc="periodic"), di.HamSpec("j1j2", "periodic"), "fp32", 3),
]


@pytest.mark.parametrize("shape,ham,prec,B", LR_CASES, ids=lambda x: str(x)[:40])
@pytest.mark.parametrize("scale", ["baseline", "stress"])
def test_logratio_and_eloc_match_oracle(L, shape, ham, prec, B, scale):
    _say("logratio", shape, ham.kind, prec, scale)
    m, th = _model(L, shape, 23, scale, prec)
    desc = ModelDesc.of(shape)
    sp = di.uniform_spins(B, shape.N, 31)
    M_max = shape.N if ham.kind == "lrtfim" else 2 * shape.N
    ref = O.eloc_plain(desc, ham, th, sp, M_max)
    ref_ab = O.abacus_logratio(desc, th, sp, ref["sites"], ref["n_conn"])
    Om = forward(desc, th, sp)["Omega"]
    # A pair exchange's ratio is the near-cancelling sum of two opposite single-flip changes,
    # so its rounding error scales with the single-flip ratios of the same sample: pair
    # ratios are checked relative to the larger of the two magnitudes.
    lr_scale = ref_ab.abs().max().item()
    if ham.kind == "j1j2":
        single = O.connected(di.HamSpec("lrtfim", shape.bc), sp)
        _, lr1 = O.plain_logratio(desc, th, sp, single[0], single[2])
        lr_scale = max(lr_scale, lr1.abs().max().item())
    spd = torch.tensor(sp, device="cuda")
    for path in ("abacus", "full"):
        lp, lr, el = m.eloc(ham, spd, M_max, path=path)
        lp, lr, el = lp.cpu(), lr.cpu(), el.cpu()
        e_lp = eps(lp, ref["logpsi"])
        e_lr = eps(lr, ref_ab)
        e_el = eps(el, ref["eloc"])
        _say(f"  {path}: eps_logpsi {e_lp:.3e} eps_lr {e_lr:.3e} eps_eloc {e_el:.3e}")
        if prec == "fp64":
            tol = 1e-10
            assert e_lp <= tol and e_el <= tol
            # the plain difference carries a rounding floor ~ eps |Omega|^2 (see module doc)
            floor = 0.0 if path == "abacus" else 1e3 * 2.2e-16 * (Om.abs().max().item() ** 2)
            assert (lr - ref_ab).abs().max().item() <= tol * lr_scale + floor
        else:
            assert e_lp <= 1e-4 and e_el <= 1e-4
            scale_lr = lr_scale
            if path == "full":
                scale_lr = max(scale_lr, Om.abs().max().item() ** 2)
            assert (lr - ref_ab).abs().max().item() <= 1e-4 * scale_lr


def test_abacus_pair_across_seam(L):
    # J1-J2 pairs that wrap the periodic seam, and the workload's zero-magnetisation spins
    shape = di.ModelShape(24, 3, 16, 4, bc="periodic")
    ham = di.HamSpec("j1j2", "periodic")
    _say("seam pairs", shape)
    m, th = _model(L, shape, 3, "stress", "fp64")
    sp = di.balanced_spins(4, 24, 8)
    sites, helem, n_conn, hdiag = O.connected(ham, sp, 48)
    spd = torch.tensor(sp, device="cuda")
    _, lr = m.logratio(spd, sites.int().cuda(), n_conn.int().cuda(), path="abacus")
    ref = O.abacus_logratio(ModelDesc.of(shape), th, sp, sites, n_conn)
    assert eps(lr.cpu(), ref) <= 1e-10


def test_abacus_rejects_wide_pairs(L):
    shape = di.ModelShape(20, 2, 8, 4, bc="open")
    m, th = _model(L, shape, 3, "stress", "fp64")
    sp = torch.tensor(di.uniform_spins(1, 20, 1), device="cuda")
    sites = torch.tensor([[[2, 9]]], dtype=torch.int32, device="cuda")
    n_conn = torch.tensor([1], dtype=torch.int32, device="cuda")
    with pytest.raises(L.DysonNetError) as ei:
        m.logratio(sp, sites, n_conn, path="abacus")
    assert ei.value.status == L.DN_EUNSUPPORTED
    # the full path takes any cluster
    _, lr = m.logratio(sp, sites, n_conn, path="full")
    spn = sp.cpu().numpy()
    _, ref = O.plain_logratio(ModelDesc.of(shape), th, spn, sites.cpu().long(), n_conn.cpu().long())
    assert eps(lr.cpu(), ref) <= 1e-10


@pytest.mark.parametrize("case", ["n_conn_high", "n_conn_negative", "site_outside", "pair_repeats", "spin_zero"])
@pytest.mark.parametrize("path", ["abacus", "full"])
def test_logratio_rejects_bad_work_lists(L, case, path):
    # the work list and the spins are validated on the device before any kernel reads them; a
    # good list after a bad one still gives the oracle's values
    shape = di.ModelShape(20, 2, 8, 4, bc="open")
    m, th = _model(L, shape, 3, "stress", "fp64")
    sp = torch.tensor(di.uniform_spins(2, 20, 1), device="cuda")
    sites = torch.tensor([[[2, -1], [5, 6]], [[7, -1], [0, -1]]], dtype=torch.int32, device="cuda")
    n_conn = torch.tensor([2, 2], dtype=torch.int32, device="cuda")
    bad_sites, bad_n, bad_sp = sites.clone(), n_conn.clone(), sp.clone()
    if case == "spin_zero":
        bad_sp[1, 11] = 0
    elif case == "n_conn_high":
        bad_n[1] = 3
    elif case == "n_conn_negative":
        bad_n[0] = -1
    elif case == "site_outside":
        bad_sites[1, 0, 0] = 20
    else:
        bad_sites[0, 1, 1] = 5
    with pytest.raises(L.DysonNetError) as ei:
        m.logratio(bad_sp, bad_sites, bad_n, path=path)
    assert ei.value.status == L.DN_EINVAL
    _, lr = m.logratio(sp, sites, n_conn, path=path)
    _, ref = O.plain_logratio(ModelDesc.of(shape), th, sp.cpu().numpy(), sites.cpu().long(), n_conn.cpu().long())
    assert eps(lr.cpu(), ref) <= 1e-10


def test_workspace_limit_gives_enomem(L):
    shape = di.ModelShape(64, 2, 32, 16, bc="open")
    m, th = _model(L, shape, 3, "baseline", "fp32")
    m.set_workspace_limit(1 << 16)
    sp = torch.tensor(di.uniform_spins(8, 64, 1), device="cuda")
    with pytest.raises(L.DysonNetError) as ei:
        m.eloc(di.HamSpec("lrtfim", "open"), sp, 64)
    assert ei.value.status == L.DN_ENOMEM


def test_empty_batch_and_state_errors(L):
    shape = di.ModelShape(16, 1, 8, 4, act="tanh")
    m = L.Model(shape, "fp64")
    sp = torch.tensor(di.uniform_spins(2, 16, 1), device="cuda")
    with pytest.raises(L.DysonNetError) as ei:
        m.logpsi(sp)
    assert ei.value.status == L.DN_ESTATE
    m.set_params(torch.tensor(di.draw_params(shape, 1, "baseline")))
    out = m.logpsi(sp[:0])
    assert out.numel() == 0


# float64 networks whose chains span several 64-site tiles, with a ragged last tile: the
# per-tile read-outs, partial slices summed across tiles, tile positions and (periodic) tap
# windows that wrap the seam, against the oracle's full re-evaluation at 1e-10.
MULTI_TILE_FP64 = [
    # shape, ham, B
    (di.ModelShape(130, 3, 32, 16, bc="open"), di.HamSpec("lrtfim", "open", alpha=2.0, h=0.5), 2),
    (di.ModelShape(130, 4, 64, 32, bc="open"), di.HamSpec("lrtfim", "open", alpha=2.0, h=0.5), 2),
    (di.ModelShape(130, 3, 64, 32, bc="periodic"), di.HamSpec("j1j2", "periodic"), 2),
    (di.ModelShape(130, 4, 32, 16, act="tanh", bc="periodic"),
     di.HamSpec("lrtfim", "periodic", J=-1.0, alpha=3.0, h=0.7, paper_form=1), 2),
    (di.ModelShape(256, 2, 64, 32, bc="open"), di.HamSpec("lrtfim", "open", alpha=2.0, h=0.5), 1),
    (di.ModelShape(200, 4, 16, 8, act="identity", bc="open"), di.HamSpec("j1j2", "open"), 2),
]


def _lr_scale(desc, ham, th, sp, ref_lr):
    """Magnitude a log-ratio error is judged against: max|lr*|, and for pair exchanges the
    larger single-flip ratios of the same samples (see the module doc)."""
    scale = ref_lr.abs().max().item()
    if ham.kind == "j1j2":
        single = O.connected(di.HamSpec("lrtfim", desc.bc), sp)
        _, lr1 = O.plain_logratio(desc, th, sp, single[0], single[2])
        scale = max(scale, lr1.abs().max().item())
    return scale


@pytest.mark.parametrize("shape,ham,B", MULTI_TILE_FP64, ids=lambda x: str(x)[:44])
def test_fp64_multi_tile_match_oracle(L, shape, ham, B):
    _say("fp64 multi-tile", shape, ham.kind)
    m, th = _model(L, shape, 29, "stress", "fp64")
    desc = ModelDesc.of(shape)
    sp = di.uniform_spins(B, shape.N, 37) if ham.kind == "lrtfim" else di.balanced_spins(B, shape.N, 37)
    M_max = shape.N if ham.kind == "lrtfim" else 2 * shape.N
    ref = O.eloc_plain(desc, ham, th, sp, M_max)
    Om = forward(desc, th, sp)["Omega"]
    lr_scale = _lr_scale(desc, ham, th, sp, ref["logratio"])
    # the oracle's own reference is a difference of two float64 evaluations
    floor = 1e3 * 2.2e-16 * max(1.0, Om.abs().max().item()) ** 2
    spd = torch.tensor(sp, device="cuda")
    for path in ("abacus", "full"):
        lp, lr, el = (t.cpu() for t in m.eloc(ham, spd, M_max, path=path))
        d_lr = (lr - ref["logratio"]).abs().max().item()
        e_lp, e_el = eps(lp, ref["logpsi"]), eps(el, ref["eloc"])
        _say(f"  {path}: eps_logpsi {e_lp:.3e} eps_eloc {e_el:.3e} |d lr| {d_lr:.3e} "
             f"(scale {lr_scale:.3e}, floor {floor:.1e})")
        assert e_lp <= 1e-10 and e_el <= 1e-10
        assert d_lr <= 1e-10 * lr_scale + floor


@pytest.mark.parametrize("name", ["tfim_n256_l4_d64", "j1j2_n128_l4_d64", "tfim_n64_l2_d32", "tfim_n256_l2_d64"])
def test_full_size_sampled(L, name):
    """Benchmark-sized batch in the benchmark's launch configuration, stress draw. The oracle
    recomputes a few samples' log-ratios one by one: ABACUS is held to them element by
    element (1e-4 of the ratio scale; ABACUS forms each change directly, so no |Omega|^2
    floor applies), and every ABACUS log-ratio of the whole batch is held to full
    re-evaluation (whose own floor is the |Omega|^2 cancellation of a difference of two
    float evaluations)."""
    w = di.WORKLOADS[name]
    shape, ham = w.model, w.ham
    B = w.B if name != "j1j2_n128_l4_d64" else 1024
    _say("full size", name, B)
    m, th = _model(L, shape, w.param_seed, "stress", "fp32")
    sp = w.spin_batch(B)
    M_max = shape.N if ham.kind == "lrtfim" else 2 * shape.N
    spd = torch.tensor(sp, device="cuda")
    lpa, lra, ela = m.eloc(ham, spd, M_max, path="abacus")
    lpf, lrf, elf = m.eloc(ham, spd, M_max, path="full")
    torch.cuda.synchronize()
    pick = [0, B // 2, B - 1]
    desc = ModelDesc.of(shape)
    ref = O.eloc_plain(desc, ham, th, sp[pick], M_max)
    Om = forward(desc, th, sp[pick])["Omega"]
    lr_scale = _lr_scale(desc, ham, th, sp[pick], ref["logratio"])
    full_floor = 1e3 * 6e-8 * max(1.0, Om.abs().max().item()) ** 2
    d_af = (lra.cpu() - lrf.cpu()).abs().max().item()
    _say(f"  abacus vs full (all {B} samples): |d lr| {d_af:.3e} (scale {lr_scale:.3e}, floor {full_floor:.1e}) "
         f"eps_eloc {eps(ela, elf):.3e}")
    assert eps(ela, elf) <= 1e-4
    assert d_af <= 1e-4 * lr_scale + full_floor
    for path, lp, lr, el in (("abacus", lpa, lra, ela), ("full", lpf, lrf, elf)):
        e_lp = eps(lp.cpu()[pick], ref["logpsi"])
        e_el = eps(el.cpu()[pick], ref["eloc"])
        d_lr = (lr.cpu()[pick] - ref["logratio"]).abs().max().item()
        bound = 1e-4 * lr_scale + (0.0 if path == "abacus" else full_floor)
        _say(f"  {path}: eps_logpsi {e_lp:.3e} eps_eloc {e_el:.3e} |d lr| {d_lr:.3e} (bound {bound:.3e})")
        assert e_lp <= 1e-4 and e_el <= 1e-4
        assert d_lr <= bound
