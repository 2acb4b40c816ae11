"""ctypes binding of libgw.so (include/gw.h): argument marshalling only.

Device arrays are torch CUDA (ROCm) float64 tensors, host arrays are NumPy.
Every computation happens in libgw.so; when the library is missing this
module raises instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgw.so")

(GW_OK, GW_ERR_ARG, GW_ERR_HIP, GW_ERR_NOMEM, GW_ERR_NOT_SPD, GW_ERR_NO_CONVERGE, GW_ERR_BLAS,
 GW_ERR_AUDIT) = range(8)
GW_FP64 = 0
GW_FP32 = 1
GW_BF16X3 = 2
PRECISIONS = {"fp64": GW_FP64, "fp32": GW_FP32, "bf16x3": GW_BF16X3}
# GW_PADE_WINDOW_HA of include/gw.h: the paper's analytic continuation window, 10 eV
PADE_WINDOW_HA = 10.0 / 27.211386245988


class GWError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libgw error {code}: {msg}")
        self.code = code


class _System(ctypes.Structure):
    _fields_ = [("n_atoms", ctypes.c_int32), ("ao_per_atom", ctypes.c_int32),
                ("ri_per_atom", ctypes.c_int32), ("n_occ", ctypes.c_int32),
                ("n_trip", ctypes.c_int64), ("trip", ctypes.c_void_p), ("t3c", ctypes.c_void_p),
                ("xyz", ctypes.c_void_p), ("ao_off", ctypes.c_void_p), ("ri_off", ctypes.c_void_p)]


class _Mlp(ctypes.Structure):
    _fields_ = [("n_features", ctypes.c_int32), ("hidden", ctypes.c_int32), ("step", ctypes.c_int32),
                ("params", ctypes.c_void_p), ("params16", ctypes.c_void_p),
                ("adam_m", ctypes.c_void_p), ("adam_v", ctypes.c_void_p), ("grad", ctypes.c_void_p)]


class _ChiOpts(ctypes.Structure):
    _fields_ = [("prec", ctypes.c_int32), ("filter_eps", ctypes.c_double), ("timing", ctypes.c_int32),
                ("screener", ctypes.c_void_p), ("screen_margin", ctypes.c_double),
                ("screen_tau", ctypes.c_void_p), ("keep_small_blocks", ctypes.c_int32),
                ("screen_audit", ctypes.c_int32), ("screen_fallback", ctypes.c_int32)]


class _ChiStats(ctypes.Structure):
    _fields_ = [("n_trip_kept", ctypes.c_int64), ("n_dblk_dropped", ctypes.c_int64),
                ("n_chiblk_dropped", ctypes.c_int64), ("flops_ab", ctypes.c_double),
                ("flops_c", ctypes.c_double), ("ms_total", ctypes.c_double),
                ("ms_stage", ctypes.c_double * 3), ("n_launch", ctypes.c_int64 * 3),
                ("flops_stage", ctypes.c_double * 3), ("n_blocks_screened", ctypes.c_int64),
                ("n_tiles_screened", ctypes.c_int64), ("c_variant", ctypes.c_int32),
                ("launch_mask", ctypes.c_int32), ("audit_done", ctypes.c_int32),
                ("audit_fallback", ctypes.c_int32), ("n_audit_violations", ctypes.c_int64),
                ("audit_max_skipped", ctypes.c_double), ("audit_skipped_mass", ctypes.c_double),
                ("audit_ms", ctypes.c_double)]


class _SigmaStats(ctypes.Structure):
    _fields_ = [("flops", ctypes.c_double), ("ms_total", ctypes.c_double)]


class _QpOpts(ctypes.Structure):
    _fields_ = [("pade_window", ctypes.c_double), ("newton_tol", ctypes.c_double),
                ("max_iter", ctypes.c_int32)]


_LIB = None
_P = ctypes.c_void_p
_I32 = ctypes.c_int32
_D = ctypes.c_double


def lib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        L.gw_build_gt.argtypes = [_P, _P, _P, _D, _I32, _P, _P, _P, _P]
        L.gw_contract_chi.argtypes = [_P, _P, _P, _I32, _P, _P, _P, _P]
        L.gw_screen_w.argtypes = [_P, _P, _P, _I32, _I32, _P, _P, _D, _P, _P]
        L.gw_contract_sigma_prec.argtypes = [_P, _I32, _P, _P, _P, _P, _P, _P, _P, _I32, _D, _I32,
                                             _P, _P, _P, _P, _P]
        L.gw_contract_sigma_prec.restype = ctypes.c_int32
        L.gw_contract_sigma.argtypes = [_P, _I32, _P, _P, _P, _P, _P, _P, _P, _I32, _D, _P, _P, _P,
                                        _P, _P]
        L.gw_continue_qp.argtypes = [_I32, _P, _P, _P, _P, _P, _P, _D, _I32, _I32, _P, _P, _P, _P,
                                     _P, _P]
        L.gw_evgw_update.argtypes = [_I32, _I32, _P, _I32, _P, _P, _P, _P]
        L.gw_fermi_level.argtypes = [_I32, _P, _P, _P, _P]
        L.gw_fermi_level.restype = ctypes.c_int32
        L.gw_screen_w_spins.argtypes = [_P, _P, _P, _P, _I32, _I32, _P, _P, _P, _P]
        L.gw_screen_w_spins.restype = ctypes.c_int32
        L.gw_screen_w_metric.argtypes = [_P, _P, _P, _P, _I32, _I32, _P, _P, _D, _P, _P, _P]
        L.gw_screen_w_metric.restype = ctypes.c_int32
        L.gw_screen_w_spins_metric.argtypes = [_P, _P, _P, _P, _P, _I32, _I32, _P, _P, _P, _P, _P]
        L.gw_screen_w_spins_metric.restype = ctypes.c_int32
        L.gw_t3c_gaussian.argtypes = [_P, _P, _P, _P, _P, _P, _P]
        L.gw_t3c_gaussian.restype = ctypes.c_int32
        L.gw_coulomb_periodic.argtypes = [_I32, _P, _P, _P, _D, _D, _P, _P, _P]
        L.gw_coulomb_periodic.restype = ctypes.c_int32
        for f in ("gw_build_gt", "gw_contract_chi", "gw_screen_w", "gw_contract_sigma",
                  "gw_continue_qp", "gw_evgw_update"):
            getattr(L, f).restype = ctypes.c_int32
        L.gw_chi_block_features.argtypes = [_P, _P, _P, _I32, _P, _D, _P, _P]
        L.gw_chi_block_lognorms.argtypes = [_P, _P, _I32, _P, _P]
        L.gw_mlp_param_count.argtypes = [_I32, _I32]
        L.gw_mlp_param_count.restype = ctypes.c_int64
        L.gw_mlp_forward.argtypes = [_P, ctypes.c_int64, _P, _P, _I32, _P]
        L.gw_mlp_gradient.argtypes = [_P, _I32, _P, _P, ctypes.c_float, _P, _P, _P]
        L.gw_mlp_train_step.argtypes = [_P, _I32, _P, _P, ctypes.c_float, ctypes.c_float, _P, _P]
        L.gw_mlp_sync_half.argtypes = [_P, _P]
        for f in ("gw_chi_block_features", "gw_chi_block_lognorms", "gw_mlp_forward",
                  "gw_mlp_gradient", "gw_mlp_train_step", "gw_mlp_sync_half"):
            getattr(L, f).restype = ctypes.c_int32
        L.gw_chi_batch_create.argtypes = [_I32, _P, _I32, _P, _P, _P]
        L.gw_chi_batch_execute.argtypes = [_P, _P, _P, _P, _I32, _P, _P]
        L.gw_chi_batch_set_config.argtypes = [_P, _I32, _I32]
        L.gw_chi_batch_set_engine.argtypes = [_P, _I32]
        L.gw_chi_batch_get_config.argtypes = [_P, _P, _P, _P]
        L.gw_chi_batch_tune.argtypes = [_P, _P, _P, _P, _I32, ctypes.c_char_p, _P, _P]
        L.gw_chi_batch_destroy.argtypes = [_P]
        for f in ("gw_chi_batch_create", "gw_chi_batch_execute", "gw_chi_batch_set_config",
                  "gw_chi_batch_set_engine", "gw_chi_batch_get_config", "gw_chi_batch_tune",
                  "gw_chi_batch_destroy"):
            getattr(L, f).restype = ctypes.c_int32
        L.gw_finalize.argtypes = []
        L.gw_finalize.restype = ctypes.c_int32
        L.gw_last_error.restype = ctypes.c_char_p
        L.gw_last_error.argtypes = []
        L.gw_version.restype = ctypes.c_char_p
        L.gw_version.argtypes = []
        _LIB = L
    return _LIB


EXPORTED = ("gw_build_gt", "gw_contract_chi", "gw_screen_w", "gw_contract_sigma",
            "gw_continue_qp", "gw_last_error", "gw_version", "gw_chi_block_features",
            "gw_chi_block_lognorms", "gw_mlp_param_count", "gw_mlp_forward", "gw_mlp_gradient",
            "gw_mlp_train_step", "gw_mlp_sync_half", "gw_chi_batch_create", "gw_chi_batch_execute",
            "gw_chi_batch_set_config", "gw_chi_batch_set_engine", "gw_chi_batch_get_config",
            "gw_chi_batch_tune", "gw_chi_batch_destroy", "gw_evgw_update", "gw_contract_sigma_prec", "gw_screen_w_spins",
            "gw_screen_w_metric", "gw_coulomb_periodic", "gw_screen_w_spins_metric",
            "gw_fermi_level", "gw_finalize", "gw_t3c_gaussian")


def _check(code):
    if code != GW_OK:
        raise GWError(code, lib().gw_last_error().decode())


def _host(a, dtype=np.float64):
    a = np.ascontiguousarray(a, dtype=dtype)
    return a, a.ctypes.data_as(ctypes.c_void_p)


def _dev(t, shape=None, dtype="float64", name="device argument"):
    """Pointer of a device tensor after checking its dtype and shape (checked
    first, so that a wrong argument raises before anything reaches the
    library), then that it is a contiguous GPU tensor."""
    if t is None:
        return None
    if dtype is not None and str(t.dtype) != "torch." + dtype:
        raise ValueError(f"{name}: dtype {t.dtype}, expected torch.{dtype}")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name}: shape {tuple(t.shape)}, expected {tuple(shape)}")
    if not (t.is_cuda and t.is_contiguous()):
        raise ValueError(f"{name}: must be a contiguous GPU tensor")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


class System:
    """A system description (gw_system) with its host triple list and device
    bricks.  ao_off / ri_off (host [n_atoms + 1], optional): per-atom function
    offsets of atoms with different numbers of functions (the bricks keep the
    per-atom maxima ao_per_atom / ri_per_atom, zeros where a function does
    not exist)."""

    def __init__(self, n_atoms, ao_per_atom, ri_per_atom, n_occ, trip, t3c, xyz=None, ao_off=None,
                 ri_off=None):
        self.trip = np.ascontiguousarray(trip, dtype=np.int32).reshape(-1, 3)
        if t3c is not None and len(self.trip):
            if str(t3c.dtype) != "torch.float64" or not t3c.is_contiguous():
                raise ValueError("t3c: contiguous float64 bricks expected")
            if t3c.numel() != len(self.trip) * ao_per_atom * ao_per_atom * ri_per_atom:
                raise ValueError(f"t3c: {t3c.numel()} elements for {len(self.trip)} bricks of "
                                 f"{ao_per_atom}x{ao_per_atom}x{ri_per_atom}")
        self.t3c = t3c
        self.xyz = None if xyz is None else np.ascontiguousarray(xyz, dtype=np.float64)
        off = lambda o: None if o is None else np.ascontiguousarray(o, dtype=np.int32)
        self.ao_off, self.ri_off = off(ao_off), off(ri_off)
        for o in (self.ao_off, self.ri_off):
            if o is not None and o.shape != (n_atoms + 1,):
                raise ValueError("per-atom offsets: n_atoms + 1 entries expected")
        ptr = lambda a: None if a is None else a.ctypes.data_as(ctypes.c_void_p).value
        self.c = _System(int(n_atoms), int(ao_per_atom), int(ri_per_atom), int(n_occ),
                         len(self.trip), self.trip.ctypes.data_as(ctypes.c_void_p).value,
                         t3c.data_ptr() if t3c is not None and len(self.trip) else None,
                         ptr(self.xyz), ptr(self.ao_off), ptr(self.ri_off))
        self.n_ao = n_atoms * ao_per_atom if self.ao_off is None else int(self.ao_off[-1])
        self.n_ri = n_atoms * ri_per_atom if self.ri_off is None else int(self.ri_off[-1])

    @property
    def ref(self):
        return ctypes.byref(self.c)


def t3c_gaussian(sys, ao_exp, ao_off, ri_exp, ri_off, t3c=None, stream=None):
    """gw_t3c_gaussian: the bricks of the system's triples (sys.trip, sys.xyz)
    as three-center overlap integrals (Eq. 4) of s-type Gaussians; returns
    the device bricks [n_trip][ao][ao][ri]."""
    import torch
    na, nr = sys.c.ao_per_atom, sys.c.ri_per_atom
    ae, ae_p = _host(ao_exp)
    re_, re_p = _host(ri_exp)
    ao_o, ao_p = _host(np.reshape(ao_off, (-1, 3)))
    ri_o, ri_p = _host(np.reshape(ri_off, (-1, 3)))
    if len(ae) != na or len(re_) != nr or ao_o.shape != (na, 3) or ri_o.shape != (nr, 3):
        raise ValueError("one exponent and offset per AO / RI function of an atom expected")
    if sys.xyz is None:
        raise ValueError("the system needs its atom coordinates")
    shape = (len(sys.trip), na, na, nr)
    if t3c is None:
        t3c = torch.empty(shape, dtype=torch.float64, device="cuda")
    _check(lib().gw_t3c_gaussian(sys.ref, ae_p, ao_p, re_p, ri_p,
                                 _dev(t3c, shape, name="t3c"), _stream(stream)))
    return t3c


def build_gt(sys, C, eps, mu_f, tau, d_occ=None, d_vir=None, stream=None):
    import torch
    tau_h, tau_p = _host(tau)
    eps_h, eps_p = _host(eps)
    n = sys.n_ao
    # None: allocate the output; False: skip that branch (NULL pointer)
    if d_occ is None:
        d_occ = torch.empty((len(tau_h), n, n), dtype=torch.float64, device=C.device)
    if d_vir is None:
        d_vir = torch.empty((len(tau_h), n, n), dtype=torch.float64, device=C.device)
    _dev(C, (n, n), name="C")
    d_occ = None if d_occ is False else d_occ
    d_vir = None if d_vir is False else d_vir
    if len(eps_h) != n:
        raise ValueError(f"eps: {len(eps_h)} energies for {n} AO functions")
    dshape = (len(tau_h), n, n)
    pc = _dev(C, (n, n), name="C")
    po, pv = _dev(d_occ, dshape, name="d_occ"), _dev(d_vir, dshape, name="d_vir")
    _check(lib().gw_build_gt(sys.ref, pc, eps_p, float(mu_f), len(tau_h), tau_p, po, pv,
                             _stream(stream)))
    return d_occ, d_vir


def contract_chi(sys, d_occ, d_vir, filter_eps=0.0, chi=None, stream=None, timing=False,
                 prec="fp64", screener=None, screen_margin=1.0, tau=None, keep_small_blocks=False,
                 audit=False, fallback=False):
    """gw_contract_chi: (chi, stats).  With a screener, audit=True judges the
    skipped blocks by the exact contraction (GWError with GW_ERR_AUDIT when one
    of them is kept by the exact filter, unless fallback=True, which returns the
    exact chi instead)."""
    import torch
    n_tau = d_occ.shape[0]
    if chi is None:
        chi = torch.empty((n_tau, sys.n_ri, sys.n_ri), dtype=torch.float64, device=d_occ.device)
    dshape, cshape = (n_tau, sys.n_ao, sys.n_ao), (n_tau, sys.n_ri, sys.n_ri)
    po, pv = _dev(d_occ, dshape, name="d_occ"), _dev(d_vir, dshape, name="d_vir")
    pchi = _dev(chi, cshape, name="chi")
    tau_h = None if tau is None else np.ascontiguousarray(tau, dtype=np.float64)
    opts = _ChiOpts(PRECISIONS[prec], float(filter_eps), int(bool(timing)),
                    None if screener is None else ctypes.addressof(screener.c),
                    float(screen_margin),
                    None if tau_h is None else tau_h.ctypes.data_as(ctypes.c_void_p).value,
                    int(bool(keep_small_blocks)), int(bool(audit)), int(bool(fallback)))
    st = _ChiStats()
    _check(lib().gw_contract_chi(sys.ref, po, pv, n_tau, ctypes.byref(opts), pchi, ctypes.byref(st),
                                 _stream(stream)))
    return chi, _stats_dict(st)


def _stats_dict(st):
    return {k: (list(getattr(st, k)) if k in ("ms_stage", "n_launch", "flops_stage")
                else getattr(st, k)) for k, _ in _ChiStats._fields_}


class ChiBatch:
    """A gw_chi_batch plan over several systems (sharing AO / RI per atom).

    The systems (and their device bricks) must outlive the plan."""

    def __init__(self, systems, n_tau, filter_eps=0.0, prec="fp64", timing=False, stream=None):
        self.systems = list(systems)
        self.n_tau = int(n_tau)
        arr = (_System * len(self.systems))(*[s.c for s in self.systems])
        self._arr = arr
        opts = _ChiOpts(PRECISIONS[prec], float(filter_eps), int(bool(timing)), None, 0.0, None)
        h = ctypes.c_void_p()
        _check(lib().gw_chi_batch_create(len(self.systems), ctypes.cast(arr, _P), self.n_tau,
                                         ctypes.byref(opts), ctypes.byref(h), _stream(stream)))
        self.h = h

    def _ptrs(self, ts):
        assert len(ts) == len(self.systems)
        return (ctypes.c_void_p * len(ts))(*[_dev(t).value for t in ts])

    def outputs(self, device="cuda"):
        import torch
        return [torch.empty((self.n_tau, s.n_ri, s.n_ri), dtype=torch.float64, device=device)
                for s in self.systems]

    def _check_shapes(self, d_occ, d_vir, chi):
        if not len(d_occ) == len(d_vir) == len(chi) == len(self.systems):
            raise ValueError("one d_occ, d_vir and chi per system expected")
        for s, o, v, c in zip(self.systems, d_occ, d_vir, chi):
            want_d = (self.n_tau, s.n_ao, s.n_ao)
            want_c = (self.n_tau, s.n_ri, s.n_ri)
            _dev(o, want_d, name="d_occ")
            _dev(v, want_d, name="d_vir")
            _dev(c, want_c, name="chi")

    def execute(self, d_occ, d_vir, chi, graph=False, stats=True, stream=None):
        self._check_shapes(d_occ, d_vir, chi)
        st = _ChiStats()
        po, pv, pc = self._ptrs(d_occ), self._ptrs(d_vir), self._ptrs(chi)
        _check(lib().gw_chi_batch_execute(self.h, po, pv, pc, int(bool(graph)),
                                          ctypes.byref(st) if stats else None, _stream(stream)))
        return _stats_dict(st) if stats else None

    def set_config(self, variant, persistent):
        """persistent: mask of stages (bit 0 A, 1 B, 2 C) launched in the persistent
        form; True means all three."""
        mask = 7 if persistent is True else int(persistent)
        _check(lib().gw_chi_batch_set_config(self.h, int(variant), mask))

    def set_engine(self, engine):
        """Engine of the half contractions: 0 direct-to-LDS where the rows allow
        it (the default), 1 register-staged; the results are bit-identical."""
        _check(lib().gw_chi_batch_set_engine(self.h, int(engine)))

    def config(self):
        v, p, n = _I32(), _I32(), _I32()
        _check(lib().gw_chi_batch_get_config(self.h, ctypes.byref(v), ctypes.byref(p),
                                             ctypes.byref(n)))
        return v.value, p.value, n.value

    def tune(self, d_occ, d_vir, chi, reps=1, cache_path=None, stream=None):
        self._check_shapes(d_occ, d_vir, chi)
        ms = _D()
        po, pv, pc = self._ptrs(d_occ), self._ptrs(d_vir), self._ptrs(chi)
        _check(lib().gw_chi_batch_tune(self.h, po, pv, pc, int(reps),
                                       None if cache_path is None else str(cache_path).encode(),
                                       ctypes.byref(ms), _stream(stream)))
        return ms.value

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            _check(lib().gw_chi_batch_destroy(self.h))
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def chi_block_features(sys, d_occ, d_vir, tau, filter_eps, feat=None, stream=None):
    import torch
    n_tau = d_occ.shape[0]
    na = sys.c.n_atoms
    if feat is None:
        feat = torch.empty((n_tau, na, na, 6), dtype=torch.float32, device=d_occ.device)
    tau_h, tau_p = _host(tau)
    if len(tau_h) != n_tau:
        raise ValueError("tau: one value per D matrix expected")
    dshape = (n_tau, sys.n_ao, sys.n_ao)
    _check(lib().gw_chi_block_features(sys.ref, _dev(d_occ, dshape, name="d_occ"),
                                       _dev(d_vir, dshape, name="d_vir"), n_tau, tau_p,
                                       float(filter_eps),
                                       _dev(feat, (n_tau, na, na, 6), "float32", "feat"),
                                       _stream(stream)))
    return feat


def chi_block_lognorms(sys, chi, out=None, stream=None):
    import torch
    n_tau = chi.shape[0]
    na = sys.c.n_atoms
    if out is None:
        out = torch.empty((n_tau, na, na), dtype=torch.float32, device=chi.device)
    _check(lib().gw_chi_block_lognorms(sys.ref, _dev(chi, (n_tau, sys.n_ri, sys.n_ri), name="chi"),
                                       n_tau, _dev(out, (n_tau, na, na), "float32", "out"),
                                       _stream(stream)))
    return out


class Mlp:
    """Device buffers of the screener network (gw_mlp)."""

    def __init__(self, n_features=6, hidden=64, params=None, device="cuda"):
        import torch
        P = int(lib().gw_mlp_param_count(n_features, hidden))
        if P < 0:
            raise GWError(GW_ERR_ARG, "unsupported network shape")
        self.P = P
        z = lambda: torch.zeros(P, dtype=torch.float32, device=device)
        self.params = z() if params is None else torch.as_tensor(
            np.asarray(params, dtype=np.float32), device=device).clone()
        self.params16 = torch.zeros(P, dtype=torch.float16, device=device)
        self.m, self.v, self.grad = z(), z(), z()
        self.loss = torch.zeros(1, dtype=torch.float32, device=device)
        self.c = _Mlp(n_features, hidden, 0, self.params.data_ptr(), self.params16.data_ptr(),
                      self.m.data_ptr(), self.v.data_ptr(), self.grad.data_ptr())
        _check(lib().gw_mlp_sync_half(ctypes.byref(self.c), _stream(None)))

    def forward(self, x, fp16=True, stream=None):
        import torch
        n = x.shape[0]
        y = torch.empty(n, dtype=torch.float32, device=x.device)
        px = _dev(x, (n, self.c.n_features), "float32", "x")
        _check(lib().gw_mlp_forward(ctypes.byref(self.c), n, px, _dev(y, dtype="float32"), int(fp16),
                                    _stream(stream)))
        return y

    def gradient(self, x, t, alpha, stream=None):
        n = x.shape[0]
        _check(lib().gw_mlp_gradient(ctypes.byref(self.c), n, _dev(x, (n, self.c.n_features),
                                                                   "float32", "x"),
                                     _dev(t, (n,), "float32", "t"), float(alpha),
                                     _dev(self.grad, dtype="float32"),
                                     _dev(self.loss, dtype="float32"), _stream(stream)))
        return self.grad, self.loss

    def train_step(self, x, t, alpha, lr, stream=None):
        n = x.shape[0]
        _check(lib().gw_mlp_train_step(ctypes.byref(self.c), n, _dev(x, (n, self.c.n_features),
                                                                      "float32", "x"),
                                       _dev(t, (n,), "float32", "t"), float(alpha), float(lr),
                                       _dev(self.loss, dtype="float32"), _stream(stream)))
        return self.loss


def screen_w(sys, chi, V, cos_w, icos_w, spin=2.0, wc=None, stream=None):
    import torch
    cw, cw_p = _host(cos_w)
    iw, iw_p = _host(icos_w)
    n_w, n_tau = cw.shape
    n = sys.n_ri
    if iw.shape != (n_tau, n_w):
        raise ValueError("icos_w must be [n_tau][n_w] for cos_w [n_w][n_tau]")
    if wc is None:
        wc = torch.empty_like(chi)
    _check(lib().gw_screen_w(sys.ref, _dev(chi, (n_tau, n, n), name="chi"),
                             _dev(V, (n, n), name="V"), n_tau, n_w, cw_p, iw_p, float(spin),
                             _dev(wc, (n_tau, n, n), name="wc"), _stream(stream)))
    return wc


def screen_w_spins(sys, chi_up, chi_dn, V, cos_w, icos_w, wc=None, stream=None):
    """gw_screen_w_spins: W^c from chi_up + chi_dn (open shell, spin factor 1)."""
    import torch
    cw, cw_p = _host(cos_w)
    iw, iw_p = _host(icos_w)
    n_w, n_tau = cw.shape
    if chi_up.shape != chi_dn.shape:
        raise ValueError("chi_up and chi_dn must have the same shape")
    n = sys.n_ri
    if wc is None:
        wc = torch.empty_like(chi_up)
    cs = (n_tau, n, n)
    _check(lib().gw_screen_w_spins(sys.ref, _dev(chi_up, cs, name="chi_up"),
                                   _dev(chi_dn, cs, name="chi_dn"), _dev(V, (n, n), name="V"),
                                   n_tau, n_w, cw_p, iw_p, _dev(wc, cs, name="wc"),
                                   _stream(stream)))
    return wc


def screen_w_metric(sys, chi, V, S_ri, cos_w, icos_w, spin=2.0, wc=None, v_tilde=True,
                    stream=None):
    """gw_screen_w_metric: (W~^c stack, V~) for the RI overlap S_ri; v_tilde
    False skips V~ (returns None for it)."""
    import torch
    cw, cw_p = _host(cos_w)
    iw, iw_p = _host(icos_w)
    n_w, n_tau = cw.shape
    n = sys.n_ri
    if tuple(chi.shape) != (n_tau, n, n) or tuple(S_ri.shape) != (n, n) or tuple(V.shape) != (n, n):
        raise ValueError("chi, V and S_ri shapes must match the system and the grids")
    if wc is None:
        wc = torch.empty_like(chi)
    vt = torch.empty_like(V) if v_tilde is True else (None if v_tilde is False else v_tilde)
    _check(lib().gw_screen_w_metric(sys.ref, _dev(chi, name="chi"), _dev(V, name="V"),
                                    _dev(S_ri, name="S_ri"), n_tau, n_w, cw_p, iw_p, float(spin),
                                    _dev(wc, (n_tau, n, n), name="wc"),
                                    _dev(vt, (n, n), name="v_tilde"), _stream(stream)))
    return wc, vt


def screen_w_spins_metric(sys, chi_up, chi_dn, V, S_ri, cos_w, icos_w, wc=None, v_tilde=True,
                          stream=None):
    """gw_screen_w_spins_metric: (W~^c, V~) from chi_up + chi_dn with the RI
    overlap S_ri (spin factor 1)."""
    import torch
    cw, cw_p = _host(cos_w)
    iw, iw_p = _host(icos_w)
    n_w, n_tau = cw.shape
    n = sys.n_ri
    if chi_up.shape != chi_dn.shape or tuple(chi_up.shape) != (n_tau, n, n) or \
            tuple(S_ri.shape) != (n, n) or tuple(V.shape) != (n, n):
        raise ValueError("chi_up, chi_dn, V and S_ri shapes must match the system and grids")
    if wc is None:
        wc = torch.empty_like(chi_up)
    vt = torch.empty_like(V) if v_tilde is True else (None if v_tilde is False else v_tilde)
    _check(lib().gw_screen_w_spins_metric(sys.ref, _dev(chi_up, name="chi_up"),
                                          _dev(chi_dn, name="chi_dn"), _dev(V, name="V"),
                                          _dev(S_ri, name="S_ri"), n_tau, n_w, cw_p, iw_p,
                                          _dev(wc, (n_tau, n, n), name="wc"),
                                          _dev(vt, (n, n), name="v_tilde"), _stream(stream)))
    return wc, vt


class _CoulombInfo(ctypes.Structure):
    _fields_ = [("eta", ctypes.c_double), ("r_cut", ctypes.c_double), ("g_cut", ctypes.c_double),
                ("n_g", ctypes.c_int32), ("n_img", ctypes.c_int32)]


def coulomb_periodic(centres, alpha, cell, eta=0.0, tol=1e-17, V=None, device="cuda",
                     stream=None):
    """gw_coulomb_periodic: (V on the device, parameters used) for Gaussian RI
    charges in an orthorhombic periodic cell."""
    import torch
    c = np.ascontiguousarray(centres, dtype=np.float64).reshape(-1, 3)
    a = np.ascontiguousarray(alpha, dtype=np.float64).ravel()
    cl = np.ascontiguousarray(cell, dtype=np.float64).ravel()
    n = len(a)
    if c.shape[0] != n or cl.shape != (3,):
        raise ValueError("centres [n][3], alpha [n] and cell [3] expected")
    if V is None:
        V = torch.empty((n, n), dtype=torch.float64, device=device)
    info = _CoulombInfo()
    _check(lib().gw_coulomb_periodic(n, c.ctypes.data_as(_P), a.ctypes.data_as(_P),
                                     cl.ctypes.data_as(_P), float(eta), float(tol),
                                     _dev(V, (n, n), name="V"),
                                     ctypes.byref(info), _stream(stream)))
    return V, {k: getattr(info, k) for k, _ in _CoulombInfo._fields_}


def contract_sigma(sys, states, C, d_occ, d_vir, d_occ0, wc, V, filter_eps=0.0, stream=None,
                   prec="fp64"):
    """prec "fp64" (gw_contract_sigma) or "fp32" (gw_contract_sigma_prec)."""
    st_h, st_p = _host(states, np.int32)
    n_gw, n_tau = len(st_h), d_occ.shape[0]
    so = np.zeros((n_gw, n_tau))
    sv = np.zeros((n_gw, n_tau))
    # d_occ0 = V = None: the exchange term is skipped (sig_x returned as None)
    sx = None if d_occ0 is None and V is None else np.zeros(n_gw)
    stats = _SigmaStats()
    N, NRI = sys.n_ao, sys.n_ri
    args = (sys.ref, n_gw, st_p, _dev(C, (N, N), name="C"),
            _dev(d_occ, (n_tau, N, N), name="d_occ"), _dev(d_vir, (n_tau, N, N), name="d_vir"),
            _dev(d_occ0, (N, N) if d_occ0 is None or d_occ0.dim() == 2 else (1, N, N),
                 name="d_occ0"),
            _dev(wc, (n_tau, NRI, NRI), name="wc"), _dev(V, (NRI, NRI), name="V"),
            n_tau, float(filter_eps))
    outs = (so.ctypes.data_as(_P), sv.ctypes.data_as(_P),
            None if sx is None else sx.ctypes.data_as(_P), ctypes.byref(stats), _stream(stream))
    if prec == "fp64":
        _check(lib().gw_contract_sigma(*args, *outs))
    else:
        _check(lib().gw_contract_sigma_prec(*args, PRECISIONS[prec], *outs))
    return so, sv, sx, {"flops": stats.flops, "ms_total": stats.ms_total}


def finalize():
    """gw_finalize: release the library's cached per-device handles."""
    _check(lib().gw_finalize())


def fermi_level(channels):
    """gw_fermi_level: mu_F of one or more channels, each (eps, n_occ)."""
    eps = [np.ascontiguousarray(e, dtype=np.float64) for e, _ in channels]
    n_mo = np.array([len(e) for e in eps], dtype=np.int32)
    n_occ = np.array([int(n) for _, n in channels], dtype=np.int32)
    ptrs = (ctypes.c_void_p * len(eps))(*[e.ctypes.data for e in eps])
    mu = ctypes.c_double(0.0)
    _check(lib().gw_fermi_level(len(eps), n_mo.ctypes.data_as(_P), n_occ.ctypes.data_as(_P),
                                ctypes.cast(ptrs, _P), ctypes.byref(mu)))
    return mu.value


def evgw_update(eps0, n_occ, states, e_qp):
    """gw_evgw_update: (energies of the next Green's function, mu_F); raises
    GWError when an occupied level ends at or above a virtual one."""
    e0, e0_p = _host(eps0)
    stt, st_p = _host(states, np.int32)
    eq, eq_p = _host(e_qp)
    out = np.zeros(len(e0))
    mu = ctypes.c_double(0.0)
    _check(lib().gw_evgw_update(len(e0), int(n_occ), e0_p, len(stt), st_p, eq_p,
                                out.ctypes.data_as(_P), ctypes.byref(mu)))
    return out, mu.value


def continue_qp(sig_occ, sig_vir, sig_x, eps_n, vxc_n, is_occ, mu_f, omega, cos_w, sin_w,
                window=PADE_WINDOW_HA, tol=1e-10, max_iter=100, raise_on_fail=False):
    """gw_continue_qp: (e_qp, status).  window: Pade nodes w_k <= window (Ha);
    the paper's 10 eV by default, <= 0 for every node."""
    so, so_p = _host(sig_occ)
    sv, sv_p = _host(sig_vir)
    sx, sx_p = _host(sig_x)
    en, en_p = _host(eps_n)
    vx, vx_p = _host(vxc_n)
    io, io_p = _host(is_occ, np.int32)
    om, om_p = _host(omega)
    cw, cw_p = _host(cos_w)
    sw, sw_p = _host(sin_w)
    n_gw, n_tau = so.shape
    e = np.zeros(n_gw)
    status = np.zeros(n_gw, dtype=np.int32)
    opts = _QpOpts(float(window), float(tol), int(max_iter))
    code = lib().gw_continue_qp(n_gw, so_p, sv_p, sx_p, en_p, vx_p, io_p, float(mu_f), n_tau,
                                len(om), om_p, cw_p, sw_p, ctypes.byref(opts),
                                e.ctypes.data_as(_P), status.ctypes.data_as(_P))
    if code not in (GW_OK, GW_ERR_NO_CONVERGE) or (raise_on_fail and code != GW_OK):
        _check(code)
    return e, status
