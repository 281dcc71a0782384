"""ctypes binding of libdysonnet.so (include/dysonnet.h): argument marshalling only.

Every function here has the name of the C entry point without the ``dn_`` prefix and
passes device pointers of torch tensors plus the current HIP stream. No arithmetic of the
method happens in Python. Loading fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdysonnet.so")

DN_OK, DN_EINVAL, DN_ENOMEM, DN_EHIP, DN_EUNSUPPORTED, DN_ESTATE = range(6)
BC = {"open": 0, "periodic": 1}
ACT = {"silu": 0, "tanh": 1, "identity": 2}
PREC = {"fp64": 0, "fp32": 1, "bf16": 2}
PATH = {"abacus": 0, "full": 1}
HAM = {"lrtfim": 0, "j1j2": 1}

# Names declared in include/dysonnet.h (checked against the shared library by the tests).
EXPORTS = ("dn_param_count", "dn_model_create", "dn_set_workspace_limit", "dn_model_set_params",
           "dn_model_get_taps", "dn_logpsi", "dn_logpsi_noalloc", "dn_connected", "dn_logratio", "dn_local_energy",
           "dn_local_energy_complex",
           "dn_eloc", "dn_grad_logpsi", "dn_autotune", "dn_set_launch_shapes", "dn_set_product_mode",
           "dn_ragged_eloc", "dn_screened_sweep", "dn_screened_sweep_adaptive", "dn_sr_update", "dn_profile_enable",
           "dn_profile_read", "dn_last_error", "dn_model_destroy")
RAGGED_MODE = {"eager": 0, "graph": 1}
PRODUCT_MODE = {"split3": 0, "fp32": 1}
KERNEL_KINDS = ("s4gen", "prep", "phi", "conv", "mix_fwd", "mix_tau", "mix_deep", "slice", "tail", "gen",
                "eloc", "other", "link")


class ModelDesc(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in
                ("N", "L", "d", "s", "d_out", "w_c", "bc", "act", "inject_phi", "prec", "complex_out", "token", "d_block")]


class HamDesc(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("bc", ctypes.c_int32), ("J", ctypes.c_double),
                ("alpha", ctypes.c_double), ("h", ctypes.c_double), ("paper_form", ctypes.c_int32),
                ("J1", ctypes.c_double), ("J2", ctypes.c_double)]


class DysonNetError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"dysonnet status {status}: {msg}")
        self.status = status


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2603_11189_amd.build` (the HIP path has no fallback)")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
        L.dn_param_count.argtypes = [ctypes.POINTER(ModelDesc)]
        L.dn_param_count.restype = i64
        L.dn_model_create.argtypes = [ctypes.POINTER(ModelDesc), ctypes.POINTER(vp)]
        L.dn_set_workspace_limit.argtypes = [vp, ctypes.c_size_t]
        L.dn_model_set_params.argtypes = [vp, vp, ctypes.c_int, vp]
        L.dn_model_get_taps.argtypes = [vp, vp, vp]
        L.dn_logpsi.argtypes = [vp, vp, i32, vp, vp]
        L.dn_logpsi_noalloc.argtypes = [vp, vp, i32, vp, vp]
        L.dn_connected.argtypes = [ctypes.POINTER(HamDesc), vp, i32, i32, i32, vp, vp, vp, vp, vp]
        L.dn_logratio.argtypes = [vp, i32, vp, i32, vp, vp, i32, vp, vp, vp]
        L.dn_local_energy.argtypes = [vp, vp, vp, vp, i32, i32, vp, vp]
        L.dn_local_energy_complex.argtypes = [vp, vp, vp, vp, i32, i32, vp, vp]
        L.dn_eloc.argtypes = [vp, i32, ctypes.POINTER(HamDesc), vp, i32, i32, vp, vp, vp, vp]
        L.dn_grad_logpsi.argtypes = [vp, vp, i32, vp, vp, vp, vp, vp]
        L.dn_autotune.argtypes = [vp, ctypes.POINTER(HamDesc), i32, ctypes.POINTER(i32), ctypes.POINTER(i64), vp]
        L.dn_set_launch_shapes.argtypes = [vp, i32, i64]
        L.dn_set_product_mode.argtypes = [vp, i32]
        L.dn_ragged_eloc.argtypes = [i32, ctypes.POINTER(vp), ctypes.POINTER(HamDesc), ctypes.POINTER(vp),
                                     ctypes.POINTER(i32), ctypes.POINTER(vp), ctypes.POINTER(vp), i32, i32, vp]
        L.dn_screened_sweep.argtypes = [vp, vp, i32, i32, i32, vp, vp, ctypes.c_double, vp, vp, vp]
        L.dn_screened_sweep_adaptive.argtypes = [vp, vp, i32, i32, i32, vp, vp, vp, vp, i32, ctypes.c_double, vp,
                                                 vp, vp]
        L.dn_sr_update.argtypes = [vp, vp, vp, vp, i32, ctypes.c_double, ctypes.c_double, i32, ctypes.c_double, vp,
                                   vp, ctypes.POINTER(i32), vp]
        L.dn_profile_enable.argtypes = [vp, ctypes.c_int]
        L.dn_profile_read.argtypes = [vp, i32, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i64),
                                      ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
        L.dn_last_error.restype = ctypes.c_char_p
        L.dn_model_destroy.argtypes = [vp]
        L.dn_model_destroy.restype = None
        for fn in ("dn_model_create", "dn_set_workspace_limit", "dn_model_set_params", "dn_model_get_taps",
                   "dn_logpsi", "dn_logpsi_noalloc", "dn_connected", "dn_logratio", "dn_local_energy",
                   "dn_local_energy_complex", "dn_eloc",
                   "dn_grad_logpsi", "dn_autotune", "dn_set_launch_shapes", "dn_set_product_mode",
                   "dn_ragged_eloc", "dn_screened_sweep", "dn_screened_sweep_adaptive", "dn_sr_update",
                   "dn_profile_enable", "dn_profile_read"):
            getattr(L, fn).restype = ctypes.c_int
        _lib = L
    return _lib


def _check(st: int):
    if st != DN_OK:
        raise DysonNetError(st, lib().dn_last_error().decode())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def make_desc(shape, prec: str = "fp32") -> ModelDesc:
    return ModelDesc(shape.N, shape.L, shape.d, shape.s, shape.d_out, shape.w_c, BC[shape.bc],
                     ACT[shape.act], shape.inject_phi, PREC[prec], getattr(shape, "complex_out", 0),
                     getattr(shape, "token", 1), getattr(shape, "d_block", 0))


def make_ham(ham) -> HamDesc:
    return HamDesc(HAM[ham.kind], BC[ham.bc], ham.J, ham.alpha, ham.h, ham.paper_form, ham.J1, ham.J2)


def param_count(shape) -> int:
    return int(lib().dn_param_count(ctypes.byref(make_desc(shape))))


class Model:
    """Owner of one dn_model handle. A complex-output model returns log psi, the log-ratios and
    E_loc as complex128 tensors (the library's (re, im) pairs)."""

    def __init__(self, shape, prec: str = "fp32"):
        self.shape, self.prec = shape, prec
        self.out_dtype = torch.complex128 if getattr(shape, "complex_out", 0) else torch.float64
        self._desc = make_desc(shape, prec)
        h = ctypes.c_void_p()
        _check(lib().dn_model_create(ctypes.byref(self._desc), ctypes.byref(h)))
        self.handle = h

    def close(self):
        if getattr(self, "handle", None):
            lib().dn_model_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_workspace_limit(self, nbytes: int):
        _check(lib().dn_set_workspace_limit(self.handle, nbytes))

    def set_params(self, params: torch.Tensor):
        """params: float64 tensor (host or device), flat, canonical order."""
        p = params.contiguous()
        assert p.dtype == torch.float64
        _check(lib().dn_model_set_params(self.handle, _ptr(p), int(p.is_cuda), _stream()))
        # which parameters the library holds (autograd checks it before a backward)
        self.param_version = getattr(self, "param_version", 0) + 1
        self.params = p.detach().clone()

    def get_taps(self) -> torch.Tensor:
        s = self.shape
        out = torch.empty((s.L + 1, s.d, 2 * s.N - 1), dtype=torch.float64, device="cuda")
        _check(lib().dn_model_get_taps(self.handle, _ptr(out), _stream()))
        return out

    def logpsi(self, spins: torch.Tensor) -> torch.Tensor:
        B = spins.shape[0]
        out = torch.empty(B, dtype=self.out_dtype, device=spins.device)
        _check(lib().dn_logpsi(self.handle, _ptr(spins), B, _ptr(out), _stream()))
        return out

    def logpsi_noalloc(self, spins: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        """dn_logpsi_noalloc: log psi with the library's scratch array (no device allocation
        inside the call; `out` may be given to avoid torch's own allocation too)."""
        B = spins.shape[0]
        if out is None:
            out = torch.empty(B, dtype=self.out_dtype, device=spins.device)
        assert out.dtype == self.out_dtype and out.is_contiguous()
        _check(lib().dn_logpsi_noalloc(self.handle, _ptr(spins), B, _ptr(out), _stream()))
        return out

    def logratio(self, spins, sites, n_conn, path: str = "abacus", want_logpsi: bool = True):
        B, M_max = sites.shape[0], sites.shape[1]
        lr = torch.empty((B, M_max), dtype=self.out_dtype, device=spins.device)
        lp = torch.empty(B, dtype=self.out_dtype, device=spins.device) if want_logpsi else None
        _check(lib().dn_logratio(self.handle, PATH[path], _ptr(spins), B, _ptr(sites), _ptr(n_conn), M_max,
                                 _ptr(lp), _ptr(lr), _stream()))
        return lp, lr

    def eloc(self, ham, spins, M_max: int, path: str = "abacus", out=None):
        B = spins.shape[0]
        if out is None:
            out = (torch.empty(B, dtype=self.out_dtype, device=spins.device),
                   torch.empty((B, M_max), dtype=self.out_dtype, device=spins.device),
                   torch.empty(B, dtype=self.out_dtype, device=spins.device))
        lp, lr, el = out
        assert all(t is None or t.dtype == self.out_dtype for t in out)
        hd = make_ham(ham)
        _check(lib().dn_eloc(self.handle, PATH[path], ctypes.byref(hd), _ptr(spins), B, M_max, _ptr(lp), _ptr(lr),
                             _ptr(el), _stream()))
        return lp, lr, el


    def grad_logpsi(self, spins: torch.Tensor, weights: torch.Tensor | None = None, want_grads: bool = True):
        """(logpsi [B], grads [B, P] or None, wsum [P] or None) of d log psi / d theta per sample.
        A complex-output model gives complex logpsi, grads (d Re + i d Im) and wsum."""
        B = spins.shape[0]
        P = param_count(self.shape)
        parts = 2 if self.out_dtype == torch.complex128 else 1
        dt = torch.float64 if self.prec == "fp64" else torch.float32
        lp = torch.empty(B, dtype=self.out_dtype, device=spins.device)
        g = torch.empty((parts, B, P), dtype=dt, device=spins.device) if want_grads else None
        ws = torch.empty((parts, P), dtype=torch.float64, device=spins.device) if weights is not None else None
        w = weights.to(torch.float64).contiguous() if weights is not None else None
        _check(lib().dn_grad_logpsi(self.handle, _ptr(spins), B, _ptr(lp), _ptr(g), _ptr(w), _ptr(ws), _stream()))
        if parts == 1:
            return lp, (g[0] if g is not None else None), (ws[0] if ws is not None else None)
        return lp, (torch.complex(g[0], g[1]) if g is not None else None), \
            (torch.complex(ws[0], ws[1]) if ws is not None else None)

    def screened_sweep(self, spins: torch.Tensor, spacing: int, parity: int, r_site: torch.Tensor,
                       u: torch.Tensor, eps: float):
        """One half-sweep of the screened typewriter sampler (dn_screened_sweep); spins are updated
        in place. Returns (accepted int32 [B, K], refreshes int32 [B])."""
        B, N = spins.shape
        K = ((N + spacing - 1) // spacing - parity + 1) // 2
        acc = torch.zeros((B, K), dtype=torch.int32, device=spins.device)
        ref = torch.zeros(B, dtype=torch.int32, device=spins.device)
        r = r_site.to(torch.float64).contiguous()
        uu = u.to(torch.float64).contiguous()
        assert r.shape == (B, K) and uu.shape == (B, K)
        _check(lib().dn_screened_sweep(self.handle, _ptr(spins), B, spacing, parity, _ptr(r), _ptr(uu), eps,
                                       _ptr(acc), _ptr(ref), _stream()))
        return acc, ref

    def screened_sweep_adaptive(self, spins: torch.Tensor, spacing: int, parity: int, r_site: torch.Tensor,
                                u: torch.Tensor, eps_buf: torch.Tensor, eps_set: torch.Tensor, gamma: float):
        """dn_screened_sweep_adaptive: the half-sweep with the tolerance buffer eps_buf (float64)
        and its flags eps_set (int32), both device tensors updated in place."""
        B, N = spins.shape
        K = ((N + spacing - 1) // spacing - parity + 1) // 2
        acc = torch.zeros((B, K), dtype=torch.int32, device=spins.device)
        ref = torch.zeros(B, dtype=torch.int32, device=spins.device)
        r = r_site.to(torch.float64).contiguous()
        uu = u.to(torch.float64).contiguous()
        assert r.shape == (B, K) and uu.shape == (B, K)
        assert eps_buf.dtype == torch.float64 and eps_set.dtype == torch.int32 and eps_buf.shape == eps_set.shape
        assert eps_buf.is_contiguous() and eps_set.is_contiguous()
        _check(lib().dn_screened_sweep_adaptive(self.handle, _ptr(spins), B, spacing, parity, _ptr(r), _ptr(uu),
                                                _ptr(eps_buf), _ptr(eps_set), eps_buf.numel(), gamma, _ptr(acc),
                                                _ptr(ref), _stream()))
        return acc, ref

    def sr_update(self, grads: torch.Tensor, eloc: torch.Tensor, weights: torch.Tensor | None = None,
                  shift: float = 1e-3, eta: float = 0.05, max_iter: int = 200, tol: float = 1e-10):
        """dn_sr_update: (delta [P] float64, energy scalar tensor, CG iterations). A complex-output
        model takes complex grads and eloc (as grad_logpsi and eloc return them) and reports a
        complex energy."""
        B, P = grads.shape
        cplx = self.out_dtype == torch.complex128
        delta = torch.empty(P, dtype=torch.float64, device=grads.device)
        energy = torch.empty(2 if cplx else 1, dtype=torch.float64, device=grads.device)
        it = ctypes.c_int32()
        w = weights.to(torch.float64).contiguous() if weights is not None else None
        if cplx:  # the library's layout: O [2][B][P] (real parts, then imaginary parts), E [B][2]
            g = torch.stack([grads.real, grads.imag]).contiguous()
            e = torch.view_as_real(eloc.to(torch.complex128).contiguous()).contiguous()
        else:
            g, e = grads.contiguous(), eloc.to(torch.float64).contiguous()
        _check(lib().dn_sr_update(self.handle, _ptr(g), _ptr(e), _ptr(w), B, shift, eta, max_iter, tol, _ptr(delta),
                                  _ptr(energy), ctypes.byref(it), _stream()))
        return delta, (torch.complex(energy[0], energy[1]) if cplx else energy[0]), it.value

    def autotune(self, ham, B_probe: int = 256):
        """Pick this model's launch shapes by timing; returns (conv_nt, flip_budget_bytes)."""
        nt, bud = ctypes.c_int32(), ctypes.c_int64()
        hd = make_ham(ham)
        _check(lib().dn_autotune(self.handle, ctypes.byref(hd), B_probe, ctypes.byref(nt), ctypes.byref(bud),
                                 _stream()))
        return nt.value, bud.value

    def set_launch_shapes(self, conv_nt: int = 0, flip_budget: int = 0):
        _check(lib().dn_set_launch_shapes(self.handle, conv_nt, flip_budget))

    def set_product_mode(self, mode: str = "split3"):
        """Float matrix-core products: "split3" (three-term bf16 splits, the default) or "fp32"."""
        _check(lib().dn_set_product_mode(self.handle, PRODUCT_MODE[mode]))

    def profile_enable(self, on: bool = True):
        _check(lib().dn_profile_enable(self.handle, int(on)))

    def profile_read(self) -> dict:
        """{kind: (total_ms, launches, flops, bytes)} for every kernel class."""
        out = {}
        for k, name in enumerate(KERNEL_KINDS):
            ms, n = ctypes.c_double(), ctypes.c_int64()
            fl, by = ctypes.c_double(), ctypes.c_double()
            _check(lib().dn_profile_read(self.handle, k, ctypes.byref(ms), ctypes.byref(n), ctypes.byref(fl),
                                         ctypes.byref(by)))
            out[name] = (ms.value, n.value, fl.value, by.value)
        return out


def connected(ham, spins: torch.Tensor, M_max: int):
    B, N = spins.shape
    dev = spins.device
    sites = torch.empty((B, M_max, 2), dtype=torch.int32, device=dev)
    helem = torch.empty((B, M_max), dtype=torch.float64, device=dev)
    n_conn = torch.empty(B, dtype=torch.int32, device=dev)
    hdiag = torch.empty(B, dtype=torch.float64, device=dev)
    hd = make_ham(ham)
    _check(lib().dn_connected(ctypes.byref(hd), _ptr(spins), B, N, M_max, _ptr(sites), _ptr(helem), _ptr(n_conn),
                              _ptr(hdiag), _stream()))
    return sites, helem, n_conn, hdiag


def local_energy(hdiag, helem, n_conn, logratio):
    """E_loc from log-ratios: float64, or complex128 for complex log-ratios."""
    B, M_max = helem.shape
    out = torch.empty(B, dtype=logratio.dtype, device=helem.device)
    fn = lib().dn_local_energy_complex if logratio.is_complex() else lib().dn_local_energy
    _check(fn(_ptr(hdiag), _ptr(helem), _ptr(n_conn), _ptr(logratio.contiguous()), B, M_max, _ptr(out), _stream()))
    return out


def ragged_eloc(models, hams, spins, logpsi, eloc, n_streams: int = 0, mode: str = "graph"):
    """Local estimator over a ragged batch in one submission (dn_ragged_eloc).

    models: list of Model (distinct); hams: HamSpec per instance; spins: int8 [B_i, N_i] device
    tensors; logpsi (list or None) and eloc: float64 [B_i] device tensors (complex128 for a
    complex-output model) written in place. In
    graph mode the submission is recorded on the first call with these exact tensors and
    replayed afterwards, so keep the tensors and refill the spins in place."""
    n = len(models)
    for i, m in enumerate(models):  # complex-output models take complex128 outputs
        assert eloc[i].dtype == m.out_dtype and (logpsi is None or logpsi[i] is None or logpsi[i].dtype == m.out_dtype)
    vp, i32 = ctypes.c_void_p, ctypes.c_int32
    mh = (vp * n)(*[m.handle for m in models])
    hd = (HamDesc * n)(*[make_ham(h) for h in hams])
    sp = (vp * n)(*[s.data_ptr() for s in spins])
    bb = (i32 * n)(*[int(s.shape[0]) for s in spins])
    lp = (vp * n)(*[t.data_ptr() if t is not None else 0 for t in logpsi]) if logpsi is not None else None
    el = (vp * n)(*[t.data_ptr() for t in eloc])
    _check(lib().dn_ragged_eloc(n, mh, hd, sp, bb, lp, el, n_streams, RAGGED_MODE[mode], _stream()))
