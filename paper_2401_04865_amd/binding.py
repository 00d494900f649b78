"""Thin ctypes binding of libpe.so (include/pe.h).

Argument marshalling only: every step of the computation runs in the HIP
library.  Device arrays are torch CUDA tensors (float64, contiguous); the
binding passes their data pointers and the current HIP stream.  Importing
this module loads the library and fails loudly if it has not been built.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpe.so")

PE_OK, PE_ERR_ARG, PE_ERR_STATE, PE_ERR_DEVICE, PE_ERR_NOMEM, PE_ERR_NOT_CONVERGED, PE_ERR_NUMERIC = range(7)
PE_FP64, PE_MIXED = 0, 1
PE_REG_GAUSSIAN, PE_REG_SHELL, PE_REG_SHELL_PAPER = 0, 1, 2
PROF_CLASSES = ["spread", "fft_z_r2c", "fft_y_fwd", "fft_x_scale", "fft_y_inv", "fft_z_c2r", "gather",
                "spmv", "pair", "krylov", "precond", "near", "matvec"]
STATUS_NAMES = {0: "PE_OK", 1: "PE_ERR_ARG", 2: "PE_ERR_STATE", 3: "PE_ERR_DEVICE", 4: "PE_ERR_NOMEM",
                5: "PE_ERR_NOT_CONVERGED", 6: "PE_ERR_NUMERIC"}


class pe_params(ctypes.Structure):
    _fields_ = [
        ("box", ctypes.c_double * 3),
        ("mesh", ctypes.c_int32 * 3),
        ("P", ctypes.c_int32),
        ("eta_c", ctypes.c_double),
        ("xi", ctypes.c_double),
        ("r_cut", ctypes.c_double),
        ("split_tol", ctypes.c_double),
        ("eps", ctypes.c_double),
        ("precision", ctypes.c_int32),
        ("reg", ctypes.c_int32),
        ("shell_radius", ctypes.c_double),
        ("gmres_restart", ctypes.c_int32),
        ("max_iters", ctypes.c_int32),
        ("rel_tol", ctypes.c_double),
        ("inner_tol", ctypes.c_double),
        ("max_refine", ctypes.c_int32),
        ("use_learned_guess", ctypes.c_int32),
        ("precond", ctypes.c_int32),
        ("rhs_fp64", ctypes.c_int32),
        ("hs_radius", ctypes.c_double),
    ]


class pe_solve_info(ctypes.Structure):
    _fields_ = [
        ("iters", ctypes.c_int32),
        ("outer_refinements", ctypes.c_int32),
        ("matvecs_fp64", ctypes.c_int32),
        ("matvecs_fp32", ctypes.c_int32),
        ("rel_residual", ctypes.c_double),
        ("rel_residual_guess", ctypes.c_double),
        ("rhs_norm", ctypes.c_double),
        ("t_rhs", ctypes.c_double),
        ("t_guess", ctypes.c_double),
        ("t_solve", ctypes.c_double),
        ("t_total", ctypes.c_double),
        ("n_hist", ctypes.c_int32),
        ("hist", ctypes.c_double * 1024),
    ]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_ if k != "hist"}
        d["hist"] = list(self.hist[: self.n_hist])
        return d


class PEError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_vp = ctypes.c_void_p
_i64 = ctypes.c_int64
_i32 = ctypes.c_int32
_u64 = ctypes.c_uint64
_dbl = ctypes.c_double

# name -> argtypes (restype is pe_status = int)
SIGNATURES = {
    "pe_default_params": [ctypes.POINTER(pe_params)],
    "pe_create": [ctypes.POINTER(pe_params), _vp, ctypes.POINTER(_vp)],
    "pe_destroy": [_vp],
    "pe_get_derived": [_vp, ctypes.POINTER(_dbl)],
    "pe_set_system": [_vp, _i64, ctypes.POINTER(_i64), _vp, _vp, _vp, _vp, _vp, _i64, _vp, _vp, _vp,
                      ctypes.POINTER(_dbl)],
    "pe_apply_potential": [_vp, _vp, _vp, _vp, _i32],
    "pe_solve_polarization": [_vp, _vp, _vp, _vp, _vp, ctypes.POINTER(pe_solve_info)],
    "pe_forces_torques": [_vp, _vp, _vp, _vp, _vp, _vp, ctypes.POINTER(_dbl)],
    "pe_apply_saddle": [_vp, _vp, _vp, _i32],
    "pe_profile_enable": [_vp, _i32],
    "pe_profile_read": [_vp, ctypes.POINTER(_dbl)],
    "pe_profile_select": [_vp, ctypes.c_uint32],
    "pe_guess_init": [_vp, _u64],
    "pe_guess_set_types": [_vp, ctypes.POINTER(_i32)],
    "pe_guess_record": [_vp, _vp],
    "pe_guess_clear": [_vp],
    "pe_guess_train": [_vp, _i32, _i32, _dbl, _u64, ctypes.POINTER(_dbl)],
    "pe_guess_predict": [_vp, _vp],
    "pe_guess_save": [_vp, ctypes.c_char_p],
    "pe_guess_load": [_vp, ctypes.c_char_p],
    "pe_bd_step": [_vp, _dbl, _dbl, _dbl, _u64, _u64, _vp, _vp, _vp, _vp],
    "pe_guess_debug": [_vp, _vp, _i32, _i64, _vp, ctypes.POINTER(_dbl)],
    "pe_guess_rows": [_vp, _vp, _i64],
    "pe_guess_add_rows": [_vp, _vp, _i64],
    "pe_bd_step_noalloc": [_vp, _dbl, _dbl, _dbl, _u64, _u64, _vp, _vp, _vp, _vp],
    "pe_grand_capacitance": [_vp, _vp, ctypes.POINTER(_dbl), ctypes.POINTER(pe_solve_info)],
    "pe_workspace_size": [_vp, _i64, _i64, _i64, ctypes.POINTER(ctypes.c_size_t)],
    "pe_set_workspace": [_vp, _vp, ctypes.c_size_t],
    "pe_workspace_info": [_vp, ctypes.POINTER(ctypes.c_size_t)],
}


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build the HIP library first "
                           "(python -c 'import __graft_entry__ as g; g.build()')")
    lib = ctypes.CDLL(path)
    for name, args in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    lib.pe_last_error.argtypes = [_vp]
    lib.pe_last_error.restype = ctypes.c_char_p
    return lib


_lib = load_library()


def lib() -> ctypes.CDLL:
    return _lib


def _check(status, ctx=None):
    if status != PE_OK:
        msg = _lib.pe_last_error(ctx)
        raise PEError(status, msg.decode() if msg else "")


def _ptr(t):
    """Device pointer of a contiguous float64 CUDA tensor (or None)."""
    if t is None:
        return None
    import torch
    if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise TypeError("expected a contiguous float64 CUDA tensor")
    return ctypes.c_void_p(t.data_ptr())


def pe_default_params() -> pe_params:
    p = pe_params()
    _check(_lib.pe_default_params(ctypes.byref(p)))
    return p


def make_params(box, mesh, **kw) -> pe_params:
    p = pe_default_params()
    b = np.broadcast_to(np.asarray(box, dtype=np.float64), (3,))
    m = np.broadcast_to(np.asarray(mesh, dtype=np.int64), (3,))
    for d in range(3):
        p.box[d] = float(b[d])
        p.mesh[d] = int(m[d])
    for k, v in kw.items():
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, v)
    return p


def _stream_handle(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


class Context:
    """A pe_context bound to one torch CUDA stream."""

    def __init__(self, params: pe_params, stream=None):
        import torch
        self.torch = torch
        self.params = params
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        h = ctypes.c_void_p()
        _check(_lib.pe_create(ctypes.byref(params), _stream_handle(self.stream), ctypes.byref(h)))
        self.h = h
        self.n_body = self.n_bead = self.n_ion = 0
        self.workspace = None   # the context's device memory: a torch uint8 tensor

    def close(self):
        if getattr(self, "h", None):
            _lib.pe_destroy(self.h)
            self.h = None
        self.workspace = None

    # ---- device workspace (torch owns the memory; the library carves it)
    def pe_workspace_size(self, n_bead, n_body, n_ion):
        out = ctypes.c_size_t()
        self._chk(_lib.pe_workspace_size(self.h, int(n_bead), int(n_body), int(n_ion), ctypes.byref(out)))
        return out.value

    def pe_set_workspace(self, tensor):
        self._chk(_lib.pe_set_workspace(self.h, ctypes.c_void_p(tensor.data_ptr()), tensor.numel()))
        self.workspace = tensor

    def pe_workspace_info(self):
        out = (ctypes.c_size_t * 4)()
        self._chk(_lib.pe_workspace_info(self.h, out))
        return dict(size=out[0], in_use=out[1], peak=out[2], need=out[3])

    def reserve(self, n_bead=None, n_body=None, n_ion=None, grow=1.0):
        """Registers a workspace of at least pe_workspace_size bytes (a new
        torch tensor when the current one is smaller; live buffers move)."""
        t = self.torch
        need = self.pe_workspace_size(self.n_bead if n_bead is None else n_bead,
                                      self.n_body if n_body is None else n_body,
                                      self.n_ion if n_ion is None else n_ion)
        have = 0 if self.workspace is None else self.workspace.numel()
        if need <= have and grow <= 1.0:
            return
        size = max(need, int(have * grow))
        size = (size + (1 << 20) - 1) >> 20 << 20
        self.pe_set_workspace(t.empty(size, dtype=t.uint8, device="cuda"))

    def _run(self, name, *args):
        """Calls an entry point; on PE_ERR_NOMEM registers a larger workspace
        and calls again (the entry points are repeatable)."""
        fn = getattr(_lib, name)
        for _ in range(8):
            st = fn(self.h, *args)
            if st != PE_ERR_NOMEM:
                return st
            self.reserve(grow=1.5)
        return st

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _chk(self, status):
        _check(status, self.h)

    # ---- thin wrappers with the C names
    def pe_get_derived(self):
        out = (ctypes.c_double * 6)()
        self._chk(_lib.pe_get_derived(self.h, out))
        return dict(xi=out[0], r_cut=out[1], eta=out[2], h=out[3], nnz=int(out[4]), ncell=int(out[5]))

    def pe_set_system(self, body_offsets, bead_pos, bead_sigma, body_center, body_quat, body_charge,
                      ion_pos, ion_charge, ion_sigma, E0):
        off = np.ascontiguousarray(np.asarray(body_offsets, dtype=np.int64))
        n_body = len(off) - 1
        n_ion = 0 if ion_charge is None else int(ion_charge.numel())
        e0 = (ctypes.c_double * 3)(*[float(v) for v in np.asarray(E0, dtype=np.float64)])
        self._keep = (bead_pos, bead_sigma, body_center, body_quat, body_charge, ion_pos, ion_charge, ion_sigma)
        self.reserve(int(off[-1]), n_body, n_ion)
        self._chk(self._run(
            "pe_set_system", n_body, off.ctypes.data_as(ctypes.POINTER(_i64)), _ptr(bead_pos), _ptr(bead_sigma),
            _ptr(body_center), _ptr(body_quat), _ptr(body_charge), n_ion, _ptr(ion_pos), _ptr(ion_charge),
            _ptr(ion_sigma), e0))
        self.n_body, self.n_bead, self.n_ion = n_body, int(off[-1]), n_ion

    def pe_apply_potential(self, charges, psi_out, field_out=None, precision=PE_FP64):
        self._chk(self._run("pe_apply_potential", _ptr(charges), _ptr(psi_out), _ptr(field_out), int(precision)))

    def pe_apply_saddle(self, x, y, precision=PE_FP64):
        self._chk(self._run("pe_apply_saddle", _ptr(x), _ptr(y), int(precision)))

    def pe_profile_enable(self, on=True):
        self._chk(self._run("pe_profile_enable", 1 if on else 0))

    def pe_profile_select(self, classes=None):
        """Record events only for the named classes (None: all)."""
        mask = 0xFFFFFFFF if classes is None else sum(1 << PROF_CLASSES.index(n) for n in classes)
        self._chk(_lib.pe_profile_select(self.h, mask))

    def pe_profile_read(self):
        """{class: (launches, total ms, work units)} for float kernels, {class + '_f64': ...} for double."""
        nc = len(PROF_CLASSES)
        out = (ctypes.c_double * (6 * nc))()
        self._chk(_lib.pe_profile_read(self.h, out))
        res = {n: (int(out[3 * i]), float(out[3 * i + 1]), float(out[3 * i + 2])) for i, n in enumerate(PROF_CLASSES)}
        res.update({n + "_f64": (int(out[3 * (nc + i)]), float(out[3 * (nc + i) + 1]), float(out[3 * (nc + i) + 2]))
                    for i, n in enumerate(PROF_CLASSES)})
        return res

    def pe_solve_polarization(self, q_init, q_out, dpsi_out, dipole_out=None, check=True):
        info = pe_solve_info()
        st = self._run("pe_solve_polarization", _ptr(q_init), _ptr(q_out), _ptr(dpsi_out), _ptr(dipole_out),
                       ctypes.byref(info))
        if check and st != PE_OK:
            self._chk(st)
        return st, info

    def pe_forces_torques(self, body_force=None, body_torque=None, body_energy=None, ion_force=None,
                          bead_force=None):
        tot = ctypes.c_double()
        self._chk(self._run("pe_forces_torques", _ptr(body_force), _ptr(body_torque), _ptr(body_energy),
                                         _ptr(ion_force), _ptr(bead_force), ctypes.byref(tot)))
        return tot.value

    def pe_guess_init(self, seed):
        self._chk(self._run("pe_guess_init", int(seed)))

    def pe_guess_set_types(self, body_type):
        t = np.ascontiguousarray(np.asarray(body_type, dtype=np.int32))
        self._chk(self._run("pe_guess_set_types", t.ctypes.data_as(ctypes.POINTER(_i32))))

    def pe_guess_record(self, q_solved):
        self._chk(self._run("pe_guess_record", _ptr(q_solved)))

    def pe_guess_clear(self):
        self._chk(self._run("pe_guess_clear"))

    def pe_guess_train(self, epochs, batch, lr, seed):
        loss = ctypes.c_double()
        self._chk(self._run("pe_guess_train", int(epochs), int(batch), float(lr), int(seed), ctypes.byref(loss)))
        return loss.value

    def pe_guess_predict(self, q_out):
        self._chk(self._run("pe_guess_predict", _ptr(q_out)))

    def pe_guess_save(self, path):
        self._chk(_lib.pe_guess_save(self.h, str(path).encode()))

    def pe_guess_load(self, path):
        self._chk(self._run("pe_guess_load", str(path).encode()))

    def pe_guess_debug(self, params=None, n_rows=0):
        """(params, grad, loss): read (params None) or set the parameters; gradient over n_rows."""
        NP = 4996
        p = np.zeros(NP, dtype=np.float32) if params is None else np.ascontiguousarray(params, dtype=np.float32)
        g = np.zeros(NP, dtype=np.float32)
        loss = ctypes.c_double()
        self._chk(self._run("pe_guess_debug", p.ctypes.data_as(ctypes.c_void_p), 0 if params is None else 1,
                                      int(n_rows), g.ctypes.data_as(ctypes.c_void_p), ctypes.byref(loss)))
        return p, g, loss.value

    def pe_guess_rows(self, n_rows):
        out = np.zeros((int(n_rows), 11), dtype=np.float32)
        self._chk(self._run("pe_guess_rows", out.ctypes.data_as(ctypes.c_void_p), int(n_rows)))
        return out

    def pe_guess_add_rows(self, rows):
        r = np.ascontiguousarray(rows, dtype=np.float32)
        assert r.ndim == 2 and r.shape[1] == 11
        self._chk(self._run("pe_guess_add_rows", r.ctypes.data_as(ctypes.c_void_p), int(r.shape[0])))

    def pe_bd_step(self, dt, kT, gamma, seed, step, bead_pos, body_center, body_quat, ion_pos):
        self._chk(self._run("pe_bd_step", float(dt), float(kT), float(gamma), int(seed), int(step),
                                  _ptr(bead_pos), _ptr(body_center), _ptr(body_quat), _ptr(ion_pos)))

    # ---- conveniences on a synthetic System (inputs module)
    def load(self, system, device="cuda"):
        """pe_set_system from an inputs.System; keeps device copies on self."""
        t = self.torch
        f = lambda a: t.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device=device)
        self.sys_dev = dict(
            bead_pos=f(system.bead_pos), bead_sigma=f(system.bead_sigma), body_center=f(system.body_center),
            body_quat=f(system.body_quat), body_charge=f(system.body_charge), ion_pos=f(system.ion_pos),
            ion_charge=f(system.ion_charge), ion_sigma=f(system.ion_sigma))
        d = self.sys_dev
        self.pe_set_system(system.body_offsets, d["bead_pos"], d["bead_sigma"], d["body_center"], d["body_quat"],
                           d["body_charge"], d["ion_pos"] if system.n_ion else None,
                           d["ion_charge"] if system.n_ion else None,
                           d["ion_sigma"] if system.n_ion else None, system.E0)
        return self

    def solve(self, q_init=None, check=True):
        t = self.torch
        q = t.empty(self.n_bead, dtype=t.float64, device="cuda")
        dpsi = t.empty(max(self.n_body, 1), dtype=t.float64, device="cuda")[: self.n_body]
        S = t.empty((max(self.n_body, 1), 3), dtype=t.float64, device="cuda")[: self.n_body]
        st, info = self.pe_solve_polarization(q_init, q, dpsi.contiguous(), S.contiguous(), check=check)
        return dict(q=q, dpsi=dpsi, dipole=S, info=info.as_dict(), status=st)

    def forces(self):
        t = self.torch
        z = lambda *s: t.zeros(s, dtype=t.float64, device="cuda")
        F, L, U = z(self.n_body, 3), z(self.n_body, 3), z(self.n_body)
        fi, fb = z(self.n_ion, 3), z(self.n_bead, 3)
        tot = self.pe_forces_torques(F, L, U, fi if self.n_ion else None, fb)
        return dict(body_force=F, body_torque=L, body_energy=U, ion_force=fi, bead_force=fb, total_energy=tot)

    def capacitance(self, want_C=True):
        """(C (4 n_body)^2 device tensor or None, eps_eff 3x3 numpy, info dict)."""
        t = self.torch
        nc = 4 * self.n_body
        C = t.empty((nc, nc), dtype=t.float64, device="cuda") if want_C else None
        eps = (ctypes.c_double * 9)()
        info = pe_solve_info()
        self._chk(self._run("pe_grand_capacitance", _ptr(C), eps, ctypes.byref(info)))
        return C, np.array(eps[:], dtype=np.float64).reshape(3, 3), info.as_dict()

    def apply(self, charges, field=False, precision=PE_FP64):
        t = self.torch
        n = self.n_bead + self.n_ion
        psi = t.empty(n, dtype=t.float64, device="cuda")
        E = t.empty((n, 3), dtype=t.float64, device="cuda") if field else None
        self.pe_apply_potential(charges, psi, E, precision)
        return psi, E
