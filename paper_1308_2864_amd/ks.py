"""Python binding of ``libks.so`` (C ABI in ``include/ks.h``).

Argument marshalling only: every function forwards to the C entry point of the same
name.  Device memory and the stream come from PyTorch (``torch.cuda``); the library
itself allocates no device memory.  If the shared library has not been built this
module raises on import, so nothing can silently run without the HIP kernels.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libks.so")

# ---- constants (mirror include/ks.h) ----------------------------------------------------
KS_OK = 0
KS_E_INVAL = -1
KS_E_NOMEM = -2
KS_E_HIP = -3
KS_E_NOT_SPD = -4
KS_E_SINGULAR = -5
KS_E_NONFINITE = -6
KS_E_NOT_CONVERGED = -7
KS_E_UNSUPPORTED = -8

KS_DISC_FD7, KS_DISC_Q1 = 0, 1
KS_PREC_FP64, KS_PREC_FP32, KS_PREC_MIXED_BF16, KS_PREC_FP32_MFMA = 0, 1, 2, 3
KS_TERM_EXT, KS_TERM_HARTREE, KS_TERM_XC, KS_TERM_ALL, KS_TERM_CORR = 1, 2, 4, 7, 8
KS_TERM_TF = 16
KS_VEXT_ERF, KS_VEXT_GNH = 0, 1
KS_HARTREE_CG, KS_HARTREE_PCG_FD = 0, 1
KS_QR, KS_WY = 0, 1
KS_BB_ALT, KS_BB1, KS_BB2 = 0, 1, 2
KS_STOP_NONE, KS_STOP_GRAD, KS_STOP_STAGNATION, KS_STOP_MAXIT, KS_STOP_ERROR = 0, 1, 2, 3, 4
KS_STOP_ENERGY = 5
PHASES = ["hartree", "xc", "hamiltonian", "gram", "gradient", "retract", "small", "density"]
KS_NPHASES = len(PHASES)
STOP_NAMES = {0: "none", 1: "grad", 2: "stagnation", 3: "maxit", 4: "error", 5: "energy"}


class ks_system_desc(C.Structure):
    _fields_ = [
        ("disc", C.c_int), ("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
        ("h", C.c_double), ("box_lo", C.c_double * 3), ("p", C.c_int), ("ld", C.c_int),
        ("occupation", C.c_double), ("n_nuclei", C.c_int),
        ("R", C.POINTER(C.c_double)), ("Z", C.POINTER(C.c_double)), ("rc", C.c_double),
        ("terms", C.c_int), ("v_ext_override", C.POINTER(C.c_double)), ("precision", C.c_int),
        ("hartree_solver", C.c_int), ("hartree_tol", C.c_double), ("hartree_maxit", C.c_int),
        ("kinetic_scale", C.c_double), ("vext_kind", C.c_int), ("hartree_bc", C.c_int),
    ]


class ks_energy(C.Structure):
    _fields_ = [
        ("total", C.c_double), ("kinetic", C.c_double), ("external", C.c_double),
        ("hartree", C.c_double), ("xc", C.c_double), ("nuclear", C.c_double),
        ("grad_norm", C.c_double), ("orth_error", C.c_double), ("hartree_iters", C.c_int),
        ("hartree_relres", C.c_double),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class ks_opt_params(C.Structure):
    _fields_ = [
        ("tau0", C.c_double), ("rho1", C.c_double), ("delta", C.c_double), ("eta", C.c_double),
        ("eps_g", C.c_double), ("max_iter", C.c_int), ("bb_rule", C.c_int),
        ("retraction", C.c_int), ("tau_min", C.c_double), ("tau_max", C.c_double),
        ("h_max", C.c_int), ("reorth_tol", C.c_double), ("stagnation_tol", C.c_double),
        ("reorth_every", C.c_int), ("energy_target", C.c_double),
    ]


class ks_result(C.Structure):
    _fields_ = [
        ("iters", C.c_int), ("nfe", C.c_int), ("backtracks", C.c_int), ("ls_fail", C.c_int),
        ("reorths", C.c_int), ("stop_reason", C.c_int), ("energy", C.c_double),
        ("grad_norm", C.c_double), ("terms", ks_energy), ("seconds", C.c_double),
        ("hartree_iters_total", C.c_longlong),
    ]


class ks_iter_info(C.Structure):
    _fields_ = [("k", C.c_int), ("nfe", C.c_int), ("backtracks", C.c_int),
                ("stop_reason", C.c_int), ("energy", C.c_double), ("grad_norm", C.c_double),
                ("tau", C.c_double), ("C", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class ks_request(C.Structure):
    _fields_ = [("id", C.c_int), ("desc", ks_system_desc), ("X0", C.c_void_p),
                ("X_out", C.c_void_p), ("params", ks_opt_params)]


class ks_completion(C.Structure):
    _fields_ = [("id", C.c_int), ("status", C.c_int), ("result", ks_result),
                ("t_submit", C.c_double), ("t_admit", C.c_double), ("t_done", C.c_double),
                ("bytes", C.c_size_t)]


class ks_phase_times(C.Structure):
    _fields_ = [("ms", C.c_double * 8), ("count", C.c_longlong * 8)]

    def as_dict(self):
        return {name: (self.ms[i], self.count[i]) for i, name in enumerate(PHASES)}


KS_TUNE_AUTO = -99
KS_HBC_ZERO, KS_HBC_MONOPOLE = 0, 1


class ks_tune_info(C.Structure):
    _fields_ = [("fd_plane_mode", C.c_int), ("hx_zrun", C.c_int), ("cached", C.c_int),
                ("n_fd", C.c_int), ("n_hx", C.c_int), ("fd_modes", C.c_int * 4),
                ("fd_us", C.c_double * 4), ("hx_zruns", C.c_int * 2), ("hx_us", C.c_double * 2)]

    def as_dict(self):
        return {"fd_plane_mode": self.fd_plane_mode, "hx_zrun": self.hx_zrun,
                "cached": bool(self.cached),
                "fd_candidates_us": {int(self.fd_modes[i]): round(self.fd_us[i], 2)
                                     for i in range(self.n_fd)},
                "hx_candidates_us": {int(self.hx_zruns[i]): round(self.hx_us[i], 2)
                                     for i in range(self.n_hx)}}


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() first")
    lib = C.CDLL(LIB_PATH)
    vp, ip, dp = C.c_void_p, C.c_int, C.POINTER(C.c_double)
    sig = {
        "ks_workspace_bytes": (C.c_size_t, [C.POINTER(ks_system_desc)]),
        "ks_create_system": (ip, [C.POINTER(ks_system_desc), vp, C.c_size_t, vp, C.POINTER(vp)]),
        "ks_destroy_system": (None, [vp]),
        "ks_default_params": (None, [C.POINTER(ks_opt_params)]),
        "ks_status_string": (C.c_char_p, [ip]),
        "ks_last_error": (C.c_char_p, [vp]),
        "ks_energy_grad": (ip, [vp, vp, vp, vp, C.POINTER(ks_energy)]),
        "ks_retract": (ip, [vp, vp, vp, C.c_double, ip, vp]),
        "ks_minimize": (ip, [vp, vp, C.POINTER(ks_opt_params), C.POINTER(ks_result)]),
        "ks_density": (ip, [vp, vp, vp]),
        "ks_hartree_solve": (ip, [vp, vp, vp, ip, C.POINTER(C.c_int), dp]),
        "ks_apply_hamiltonian": (ip, [vp, vp, vp, vp]),
        "ks_get_potentials": (ip, [vp, vp, vp, vp]),
        "ks_gram": (ip, [vp, vp, vp, vp]),
        "ks_gram_static": (ip, [vp, vp, ip, ip, ip, ip, vp, vp]),
        "ks_enable_timers": (ip, [vp, ip]),
        "ks_read_timers": (ip, [vp, C.POINTER(ks_phase_times), ip]),
        "ks_enable_graphs": (ip, [vp, ip]),
        "ks_minimize_batch": (ip, [C.POINTER(vp), ip, C.POINTER(vp), C.POINTER(ks_opt_params),
                                   C.POINTER(ks_result), C.POINTER(ip)]),
        "ks_minimize_begin": (ip, [vp, vp, C.POINTER(ks_opt_params), C.POINTER(ks_iter_info)]),
        "ks_minimize_step": (ip, [vp, C.POINTER(ks_iter_info)]),
        "ks_minimize_end": (ip, [vp, vp, C.POINTER(ks_result)]),
        "ks_state_bytes": (C.c_size_t, [vp]),
        "ks_get_state": (ip, [vp, vp]),
        "ks_set_state": (ip, [vp, vp]),
        "ks_batch_step": (ip, [C.POINTER(vp), ip, C.POINTER(ks_iter_info)]),
        "ks_prolong": (ip, [vp, vp, vp, vp]),
        "ks_autotune": (ip, [vp, ip, C.POINTER(ks_tune_info)]),
        "ks_minimize_levels": (ip, [C.POINTER(vp), ip, C.POINTER(vp), C.POINTER(ks_opt_params),
                                    C.POINTER(ks_result)]),
        "ks_timer_phases": (ip, [vp, C.c_uint]),
        "ks_server_create": (ip, [vp, C.c_size_t, ip, C.POINTER(vp)]),
        "ks_server_create_batched": (ip, [vp, C.c_size_t, ip, C.POINTER(vp)]),
        "ks_server_submit": (ip, [vp, C.POINTER(ks_request)]),
        "ks_server_poll": (ip, [vp, C.POINTER(ks_completion), ip, C.POINTER(ip)]),
        "ks_server_wait_idle": (ip, [vp]),
        "ks_server_pending": (ip, [vp]),
        "ks_server_destroy": (None, [vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


lib = _load()


class KSError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{lib.ks_status_string(code).decode()} ({code}): {msg}")
        self.code = code


def _ptr(t):
    """Device pointer of a torch tensor (or None)."""
    if t is None:
        return None
    return C.c_void_p(t.data_ptr())


def _addr(buf):
    """Address of a numpy array (host) or torch tensor (device or host)."""
    if isinstance(buf, np.ndarray):
        return buf.ctypes.data
    return buf.data_ptr()


def _check(code, handle=None):
    if code != KS_OK:
        raise KSError(code, lib.ks_last_error(handle).decode(errors="replace"))
    return code


# ---- thin wrappers with the ABI's names ---------------------------------------------------

def ks_default_params(**overrides) -> ks_opt_params:
    o = ks_opt_params()
    lib.ks_default_params(C.byref(o))
    for k, v in overrides.items():
        setattr(o, k, v)
    return o


def make_desc(nx, ny, nz, h, lo, p, R=None, Z=None, *, f=2.0, rc=0.5, terms=KS_TERM_ALL,
              v_ext_override=None, ld=0, precision=KS_PREC_FP64, disc=KS_DISC_FD7,
              hartree_solver=KS_HARTREE_CG, hartree_tol=0.0, hartree_maxit=0,
              kinetic_scale=0.0, vext_kind=KS_VEXT_ERF, hartree_bc=0):
    """Fills a ks_system_desc; the returned object keeps the host arrays alive."""
    d = ks_system_desc()
    d.disc, d.nx, d.ny, d.nz, d.h = disc, nx, ny, nz, float(h)
    d.box_lo[:] = [float(v) for v in lo]
    d.p, d.ld, d.occupation = p, ld, float(f)
    R = np.ascontiguousarray(np.zeros((0, 3)) if R is None else R, dtype=np.float64).reshape(-1, 3)
    Z = np.ascontiguousarray(np.zeros(0) if Z is None else Z, dtype=np.float64).ravel()
    d.n_nuclei = int(R.shape[0])
    d._keep = [R, Z]
    d.R = R.ctypes.data_as(C.POINTER(C.c_double)) if R.size else None
    d.Z = Z.ctypes.data_as(C.POINTER(C.c_double)) if Z.size else None
    d.rc, d.terms = float(rc), int(terms)
    if v_ext_override is not None:
        v = np.ascontiguousarray(v_ext_override, dtype=np.float64).ravel()
        d._keep.append(v)
        d.v_ext_override = v.ctypes.data_as(C.POINTER(C.c_double))
    d.precision, d.hartree_solver = precision, hartree_solver
    d.hartree_tol, d.hartree_maxit = float(hartree_tol), int(hartree_maxit)
    d.kinetic_scale, d.vext_kind = float(kinetic_scale), int(vext_kind)
    d.hartree_bc = int(hartree_bc)
    return d


def ks_workspace_bytes(desc) -> int:
    return int(lib.ks_workspace_bytes(C.byref(desc)))


class KSSystem:
    """A system created by ks_create_system on a torch-owned workspace and stream."""

    def __init__(self, desc, device="cuda", stream=None):
        import torch
        self.desc = desc
        nbytes = ks_workspace_bytes(desc)
        if nbytes == 0:
            raise KSError(KS_E_INVAL, lib.ks_last_error(None).decode())
        self.device = torch.device(device)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self.workspace.data_ptr()
        off = (-base) % 256
        self.stream = stream or torch.cuda.current_stream(self.device)
        h = C.c_void_p()
        _check(lib.ks_create_system(C.byref(desc), C.c_void_p(base + off), nbytes,
                                    C.c_void_p(self.stream.cuda_stream), C.byref(h)))
        self.h = h
        self.n = desc.nx * desc.ny * desc.nz
        self.p = desc.p
        self.ld = desc.ld or desc.p

    def close(self):
        if getattr(self, "h", None):
            lib.ks_destroy_system(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # each method is one C call
    def ks_energy_grad(self, X, G=None, gradE=None) -> ks_energy:
        e = ks_energy()
        _check(lib.ks_energy_grad(self.h, _ptr(X), _ptr(G), _ptr(gradE), C.byref(e)), self.h)
        return e

    def ks_retract(self, X, G, tau, kind, X_out):
        _check(lib.ks_retract(self.h, _ptr(X), _ptr(G), float(tau), int(kind), _ptr(X_out)), self.h)

    def ks_minimize(self, X, params=None, check=True) -> ks_result:
        r = ks_result()
        code = lib.ks_minimize(self.h, _ptr(X), C.byref(params) if params is not None else None,
                               C.byref(r))
        if check and code not in (KS_OK, KS_E_NOT_CONVERGED):
            _check(code, self.h)
        r.code = code
        return r

    def ks_minimize_begin(self, X0, params=None) -> ks_iter_info:
        info = ks_iter_info()
        _check(lib.ks_minimize_begin(self.h, _ptr(X0),
                                     C.byref(params) if params is not None else None,
                                     C.byref(info)), self.h)
        return info

    def ks_minimize_step(self) -> ks_iter_info:
        info = ks_iter_info()
        _check(lib.ks_minimize_step(self.h, C.byref(info)), self.h)
        return info

    def ks_minimize_end(self, X_out=None, check=True) -> ks_result:
        r = ks_result()
        code = lib.ks_minimize_end(self.h, _ptr(X_out), C.byref(r))
        if check and code not in (KS_OK, KS_E_NOT_CONVERGED):
            _check(code, self.h)
        r.code = code
        return r

    def ks_state_bytes(self) -> int:
        return int(lib.ks_state_bytes(self.h))

    def ks_get_state(self, buf):
        """buf: a host numpy uint8 array or a device torch uint8 tensor of ks_state_bytes()."""
        _check(lib.ks_get_state(self.h, C.c_void_p(_addr(buf))), self.h)

    def ks_set_state(self, buf):
        _check(lib.ks_set_state(self.h, C.c_void_p(_addr(buf))), self.h)

    def ks_autotune(self, force=False) -> dict:
        """Times the candidate launch shapes on this system and keeps the fastest (see
        include/ks.h); returns the choice and the timings."""
        t = ks_tune_info()
        _check(lib.ks_autotune(self.h, int(bool(force)), C.byref(t)), self.h)
        return t.as_dict()

    def ks_density(self, X, rho):
        _check(lib.ks_density(self.h, _ptr(X), _ptr(rho)), self.h)

    def ks_hartree_solve(self, rho, v_h, warm=False):
        it = C.c_int()
        rr = C.c_double()
        _check(lib.ks_hartree_solve(self.h, _ptr(rho), _ptr(v_h), int(bool(warm)), C.byref(it),
                                    C.byref(rr)), self.h)
        return it.value, rr.value

    def ks_apply_hamiltonian(self, X, Y, v_eff=None):
        _check(lib.ks_apply_hamiltonian(self.h, _ptr(X), _ptr(Y), _ptr(v_eff)), self.h)

    def ks_get_potentials(self, v_ext=None, v_h=None, v_eff=None):
        _check(lib.ks_get_potentials(self.h, _ptr(v_ext), _ptr(v_h), _ptr(v_eff)), self.h)

    def ks_gram(self, A, B, out):
        _check(lib.ks_gram(self.h, _ptr(A), _ptr(B), _ptr(out)), self.h)

    def ks_enable_graphs(self, on=True):
        _check(lib.ks_enable_graphs(self.h, int(bool(on))), self.h)

    def ks_timer_phases(self, names):
        mask = 0
        for nm in names:
            mask |= 1 << PHASES.index(nm)
        _check(lib.ks_timer_phases(self.h, mask), self.h)

    def ks_enable_timers(self, on=True):
        _check(lib.ks_enable_timers(self.h, int(bool(on))), self.h)

    def ks_read_timers(self, reset=False) -> dict:
        t = ks_phase_times()
        _check(lib.ks_read_timers(self.h, C.byref(t), int(bool(reset))), self.h)
        return t.as_dict()


def desc_from_spec(spec, **kw):
    """A ks_system_desc for a ``synth.SystemSpec`` (keyword arguments go to make_desc)."""
    terms = (KS_TERM_EXT if spec.ext else 0) | (KS_TERM_HARTREE if spec.hartree else 0) | \
            (KS_TERM_XC if spec.xc else 0) | (KS_TERM_CORR if spec.corr else 0) | \
            (KS_TERM_TF if spec.tf else 0)
    dkw = dict(f=spec.f, rc=spec.rc, terms=terms,
               disc=KS_DISC_Q1 if spec.disc == "q1" else KS_DISC_FD7,
               kinetic_scale=spec.mu,
               vext_kind=KS_VEXT_GNH if spec.vext == "gnh" else KS_VEXT_ERF,
               hartree_bc=KS_HBC_MONOPOLE if spec.hartree_bc == "monopole" else KS_HBC_ZERO)
    dkw.update(kw)
    return make_desc(spec.nx, spec.ny, spec.nz, spec.h, spec.lo, spec.p, spec.R, spec.Z, **dkw)


def system_from_spec(spec, **kw) -> KSSystem:
    """Creates a KSSystem for a ``synth.SystemSpec``."""
    device = kw.pop("device", "cuda")
    return KSSystem(desc_from_spec(spec, **kw), device=device)


def ks_minimize_batch(systems, blocks, params=None):
    """ks_minimize on several KSSystem objects in lockstep (see include/ks.h).  Returns
    (list of ks_result, list of return codes)."""
    n = len(systems)
    hs = (C.c_void_p * n)(*[s.h for s in systems])
    xs = (C.c_void_p * n)(*[X.data_ptr() for X in blocks])
    rs = (ks_result * n)()
    codes = (C.c_int * n)()
    rc = lib.ks_minimize_batch(hs, n, xs, C.byref(params) if params is not None else None, rs,
                               codes)
    if rc in (KS_E_INVAL, KS_E_HIP):  # the batch itself failed; per-system codes otherwise
        _check(rc)
    return list(rs), list(codes)


def ks_gram_static(A, B, out, stream=None):
    """[A^T A, A^T B, B^T B] of two device n x p blocks into out (3 x p x p doubles) with the
    library's static scratch (no allocation; see include/ks.h).  Enqueues on the stream."""
    import torch
    if A.shape != B.shape or A.dim() != 2 or A.dtype != B.dtype:
        raise ValueError("A and B must be n x p blocks of one dtype")
    n, p = A.shape
    prec = KS_PREC_FP64 if A.dtype == torch.float64 else KS_PREC_FP32
    st = stream or torch.cuda.current_stream(A.device)
    _check(lib.ks_gram_static(_ptr(A), _ptr(B), int(n), int(p), int(A.stride(0)), prec,
                              _ptr(out), C.c_void_p(st.cuda_stream)))


def ks_batch_step(systems):
    """One lockstep trial for every listed KSSystem with a run begun (see include/ks.h).
    Returns the list of ks_iter_info."""
    n = len(systems)
    hs = (C.c_void_p * n)(*[s.h for s in systems])
    infos = (ks_iter_info * n)()
    _check(lib.ks_batch_step(hs, n, infos))
    return list(infos)


def ks_prolong(coarse, Xc, fine, Xf):
    """Carries a coarse block over to the uniformly refined system (Alg. 4; see
    include/ks.h): Xf receives the interpolated, orthonormalised block."""
    _check(lib.ks_prolong(coarse.h, _ptr(Xc), fine.h, _ptr(Xf)), fine.h)


def ks_minimize_levels(systems, blocks, params=None):
    """Alg. 4 with uniform refinement over nested KSSystem objects, coarsest first (see
    include/ks.h): blocks[0] is the start (in/out), blocks[i] receive each level's result.
    Returns the list of per-level ks_result; raises on errors other than max_iter."""
    n = len(systems)
    hs = (C.c_void_p * n)(*[s.h for s in systems])
    xs = (C.c_void_p * n)(*[X.data_ptr() for X in blocks])
    rs = (ks_result * n)()
    rc = lib.ks_minimize_levels(hs, n, xs, C.byref(params) if params is not None else None, rs)
    if rc not in (KS_OK, KS_E_NOT_CONVERGED):
        _check(rc)  # the message of the failing level (the calling thread's last error)
    return list(rs)


def ks_request_bytes(desc) -> int:
    """Device bytes a server request for desc holds while it runs (256-byte regions)."""
    desc = ks_system_desc.from_buffer_copy(desc)
    desc.ld = 0
    ws = ks_workspace_bytes(desc)
    if ws == 0:
        raise KSError(KS_E_INVAL, lib.ks_last_error(None).decode())
    es = 4 if desc.precision in (KS_PREC_FP32, KS_PREC_MIXED_BF16, KS_PREC_FP32_MFMA) else 8
    x = desc.nx * desc.ny * desc.nz * desc.p * es  # the server keeps blocks dense
    return (ws + 255) // 256 * 256 + (x + 255) // 256 * 256


class KSServer:
    """ks_server_* over a torch-owned device workspace of ``nbytes``.  With batched=True,
    n_slots is the number of requests the continuous-batching engine keeps resident.

    ``submit`` takes a descriptor, a host start block (n x p, float64 or float32 to match
    the descriptor's precision) and optional parameters; the result block, when asked
    for, is written into a host array this object keeps alive until its completion has
    been polled.
    """

    def __init__(self, nbytes, n_slots, device="cuda", batched=False):
        import torch
        self.device = torch.device(device)
        self.workspace = torch.empty(int(nbytes) + 256, dtype=torch.uint8, device=self.device)
        torch.cuda.synchronize(self.device)
        base = self.workspace.data_ptr()
        off = (-base) % 256
        h = C.c_void_p()
        create = lib.ks_server_create_batched if batched else lib.ks_server_create
        _check(create(C.c_void_p(base + off), int(nbytes), int(n_slots), C.byref(h)))
        self.h = h
        self._out = {}

    def ks_server_submit(self, rid, desc, X0, params=None, want_X=False):
        dt = np.float32 if desc.precision in (KS_PREC_FP32, KS_PREC_MIXED_BF16, KS_PREC_FP32_MFMA) else np.float64
        X0 = np.ascontiguousarray(X0, dtype=dt)
        n = desc.nx * desc.ny * desc.nz
        if X0.shape != (n, desc.p):
            raise ValueError(f"X0 must be {n} x {desc.p}")
        rq = ks_request()
        rq.id = int(rid)
        rq.desc = desc
        rq.X0 = X0.ctypes.data
        if want_X:
            out = np.empty_like(X0)
            self._out[int(rid)] = out
            rq.X_out = out.ctypes.data
        rq.params = params if params is not None else ks_default_params()
        _check(lib.ks_server_submit(self.h, C.byref(rq)))

    def ks_server_poll(self, max_n=1024):
        buf = (ks_completion * max_n)()
        k = C.c_int()
        _check(lib.ks_server_poll(self.h, buf, int(max_n), C.byref(k)))
        out = []
        for c in buf[:k.value]:
            out.append(dict(id=c.id, status=c.status, result=c.result, t_submit=c.t_submit,
                            t_admit=c.t_admit, t_done=c.t_done, bytes=int(c.bytes),
                            X=self._out.pop(c.id, None)))
        return out

    def ks_server_wait_idle(self):
        _check(lib.ks_server_wait_idle(self.h))

    def ks_server_pending(self) -> int:
        return int(lib.ks_server_pending(self.h))

    def close(self):
        if getattr(self, "h", None):
            lib.ks_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
