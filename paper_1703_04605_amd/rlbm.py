"""Thin ctypes binding of librlbm.so (the C ABI declared in include/rlbm.h).

Argument marshalling only: every step of the relativistic lattice Boltzmann
time step runs in the library's HIP kernels.  PyTorch provides device memory
(population and field buffers) and the HIP stream.  If the library is not
built, loading fails loudly; there is no fallback.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librlbm.so")

RLBM_OK = 0
RLBM_EINVAL = -1
RLBM_ENOSTENCIL = -2
RLBM_EHIP = -3
RLBM_ENUMERIC = -4
RLBM_ESTATE = -5

PRECISION = {"fp64": 0, "fp32": 1, "fp16": 2}
LANDAU = {"newton": 0, "fixed_point": 1}
BC = {"periodic": 0, "outflow": 1}
TAU_CONST, TAU_ETA_OVER_S = 0, 1
ELEM_DTYPE = {"fp64": "float64", "fp32": "float32", "fp16": "float16"}

H_NAN, H_LANDAU, H_SUPERLUMINAL, H_RANGE, H_EOS, H_SYNC = 1, 2, 4, 8, 16, 32

EXPORTS = ["rlbm_init_stencil", "rlbm_solve_stencil", "rlbm_class_table", "rlbm_destroy",
           "rlbm_population_bytes", "rlbm_init_fields", "rlbm_step", "rlbm_moments",
           "rlbm_get_health", "rlbm_step_count", "rlbm_save_state", "rlbm_load_state",
           "rlbm_last_error", "rlbm_eos_temperature_host", "rlbm_mlp_create", "rlbm_mlp_destroy",
           "rlbm_mlp_train_step", "rlbm_mlp_predict", "rlbm_mlp_get_params", "rlbm_set_landau_guess",
           "rlbm_set_warm_start",
           "rlbm_landau_guess_fields", "rlbm_batch_create", "rlbm_batch_destroy", "rlbm_batch_population_bytes",
           "rlbm_batch_sites", "rlbm_batch_init", "rlbm_batch_step_persistent", "rlbm_batch_moments",
           "rlbm_batch_get_health", "rlbm_set_step_variant", "rlbm_step_kernel", "rlbm_check_lattice",
           "rlbm_init_fields_noalloc", "rlbm_batch_occupancy", "rlbm_population_bytes3", "rlbm_init_fields3",
           "rlbm_moments3", "rlbm_device_copy"]

STEP_AUTO, STEP_TABLE, STEP_FIXED = 0, 1, 2


class RlbmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"rlbm error {code}: {msg}")
        self.code = code


class StencilDesc(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("n_groups", ctypes.c_int),
                ("group_base", ctypes.POINTER(ctypes.c_int)), ("zeta", ctypes.c_double),
                ("v0", ctypes.c_double), ("v0_lo", ctypes.c_double), ("v0_hi", ctypes.c_double),
                ("precision", ctypes.c_int), ("n_ref", ctypes.c_double), ("T_ref", ctypes.c_double),
                ("order", ctypes.c_int), ("weights", ctypes.POINTER(ctypes.c_double))]


class StencilInfo(ctypes.Structure):
    _fields_ = [("q3", ctypes.c_int), ("q", ctypes.c_int), ("v0", ctypes.c_double),
                ("v0_lo", ctypes.c_double), ("v0_hi", ctypes.c_double),
                ("weights", ctypes.c_double * 16), ("ortho_residual", ctypes.c_double),
                ("max_shift", ctypes.c_int), ("cond", ctypes.c_double)]


class LatticeDesc(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("bc_x", ctypes.c_int), ("bc_y", ctypes.c_int),
                ("tau_mode", ctypes.c_int), ("tau", ctypes.c_double), ("eta_over_s", ctypes.c_double),
                ("T_R_GeV", ctypes.c_double), ("n_unit_fm3", ctypes.c_double), ("dx_fm", ctypes.c_double),
                ("landau_tol", ctypes.c_double), ("landau_maxit", ctypes.c_int), ("landau_method", ctypes.c_int),
                ("nz", ctypes.c_int), ("bc_z", ctypes.c_int)]


class Problem(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("stencil", ctypes.c_int), ("eta_over_s", ctypes.c_double),
                ("T_R_GeV", ctypes.c_double), ("n_unit_fm3", ctypes.c_double), ("dx_fm", ctypes.c_double)]


_lib = None


def lib():
    """Loads librlbm.so (built by __graft_entry__.build()); raises if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built: run __graft_entry__.build() (no CPU fallback exists)")
    L = ctypes.CDLL(LIB_PATH)
    vp, cd, ci = ctypes.c_void_p, ctypes.c_double, ctypes.c_int
    dp = ctypes.POINTER(ctypes.c_double)
    L.rlbm_init_stencil.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(StencilDesc), ctypes.POINTER(StencilInfo)]
    L.rlbm_solve_stencil.argtypes = [ctypes.POINTER(StencilDesc), ctypes.POINTER(StencilInfo)]
    L.rlbm_class_table.argtypes = [ctypes.POINTER(StencilDesc), ci, ctypes.POINTER(ctypes.c_int), dp, dp]
    L.rlbm_destroy.argtypes = [vp]
    L.rlbm_population_bytes.argtypes = [vp, ci, ci]
    L.rlbm_population_bytes.restype = ctypes.c_size_t
    L.rlbm_init_fields.argtypes = [vp, ctypes.POINTER(LatticeDesc), vp, vp, vp, vp, vp, vp, ctypes.c_size_t, vp]
    L.rlbm_init_fields_noalloc.argtypes = [vp, ctypes.POINTER(LatticeDesc), vp, vp, vp, vp, vp, vp,
                                           ctypes.c_size_t, vp]
    L.rlbm_check_lattice.argtypes = [ctypes.POINTER(StencilDesc), ctypes.POINTER(LatticeDesc)]
    L.rlbm_population_bytes3.argtypes = [vp, ci, ci, ci]
    L.rlbm_population_bytes3.restype = ctypes.c_size_t
    L.rlbm_init_fields3.argtypes = [vp, ctypes.POINTER(LatticeDesc), vp, vp, vp, vp, vp, vp, vp, ctypes.c_size_t, vp]
    L.rlbm_moments3.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
    L.rlbm_device_copy.argtypes = [vp, vp, ctypes.c_size_t, ci, vp]
    L.rlbm_step.argtypes = [vp, ci, vp]
    L.rlbm_moments.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp]
    L.rlbm_get_health.argtypes = [vp, ctypes.POINTER(ctypes.c_uint), ctypes.POINTER(ctypes.c_ulonglong),
                                  ctypes.POINTER(ctypes.c_uint), ci, vp]
    L.rlbm_step_count.argtypes = [vp]
    L.rlbm_step_count.restype = ctypes.c_longlong
    L.rlbm_set_step_variant.argtypes = [vp, ci]
    L.rlbm_set_step_variant.restype = ci
    L.rlbm_step_kernel.argtypes = [vp]
    L.rlbm_step_kernel.restype = ci
    L.rlbm_save_state.argtypes = [vp, vp, ctypes.c_size_t, ctypes.POINTER(ctypes.c_longlong),
                                  ctypes.POINTER(ctypes.c_int), vp]
    L.rlbm_load_state.argtypes = [vp, vp, ctypes.c_size_t, ctypes.c_longlong, ci, vp]
    L.rlbm_eos_temperature_host.argtypes = [cd, dp, ci, dp]
    fp = ctypes.POINTER(ctypes.c_float)
    L.rlbm_mlp_create.argtypes = [ctypes.POINTER(vp), fp, fp, ci]
    L.rlbm_mlp_destroy.argtypes = [vp]
    L.rlbm_mlp_train_step.argtypes = [vp, vp, vp, ci, ctypes.c_float, fp, vp]
    L.rlbm_mlp_predict.argtypes = [vp, vp, ci, vp, vp]
    L.rlbm_mlp_get_params.argtypes = [vp, fp, fp]
    L.rlbm_set_landau_guess.argtypes = [vp, vp]
    L.rlbm_set_warm_start.argtypes = [vp, ci]
    L.rlbm_landau_guess_fields.argtypes = [vp, vp, vp]
    L.rlbm_batch_create.argtypes = [ctypes.POINTER(vp), ci, ctypes.POINTER(vp), ci, ctypes.POINTER(Problem), cd, ci]
    L.rlbm_batch_destroy.argtypes = [vp]
    L.rlbm_batch_population_bytes.argtypes = [vp]
    L.rlbm_batch_population_bytes.restype = ctypes.c_size_t
    L.rlbm_batch_sites.argtypes = [vp]
    L.rlbm_batch_sites.restype = ctypes.c_longlong
    L.rlbm_batch_init.argtypes = [vp, vp, vp, vp, vp, vp, ctypes.c_size_t, vp]
    L.rlbm_batch_step_persistent.argtypes = [vp, ci, ci, vp, vp]
    L.rlbm_batch_moments.argtypes = [vp, vp, vp, vp, vp, vp, vp]
    L.rlbm_batch_occupancy.argtypes = [vp, ctypes.POINTER(ci), ctypes.POINTER(ci), ctypes.POINTER(ci)]
    L.rlbm_batch_get_health.argtypes = [vp, ctypes.POINTER(ctypes.c_uint), ctypes.POINTER(ctypes.c_ulonglong),
                                        ctypes.POINTER(ctypes.c_uint), vp]
    L.rlbm_last_error.argtypes = [vp]
    L.rlbm_last_error.restype = ctypes.c_char_p
    _lib = L
    return L


def _check(rc, ctx=None):
    if rc != RLBM_OK:
        msg = lib().rlbm_last_error(ctx)
        raise RlbmError(rc, msg.decode() if msg else "")


def make_desc(bases, zeta, v0=0.0, dim=2, precision="fp64", n_ref=1.0, T_ref=1.0, v0_lo=0.0, v0_hi=0.0,
              order=2, weights=None):
    flat = [int(c) for b in bases for c in b]
    arr = (ctypes.c_int * len(flat))(*flat)
    warr = None if weights is None else (ctypes.c_double * len(weights))(*[float(w) for w in weights])
    d = StencilDesc(dim, len(bases), ctypes.cast(arr, ctypes.POINTER(ctypes.c_int)), float(zeta), float(v0),
                    float(v0_lo), float(v0_hi), PRECISION[precision], float(n_ref), float(T_ref), int(order),
                    None if warr is None else ctypes.cast(warr, ctypes.POINTER(ctypes.c_double)))
    d._keep = (arr, warr)
    return d


def lattice_desc(nx, ny, bc=("periodic", "periodic"), tau=1.0, landau_tol=0.0, landau_maxit=0, landau="newton"):
    if isinstance(tau, dict):
        return LatticeDesc(nx, ny, BC[bc[0]], BC[bc[1]], TAU_ETA_OVER_S, 0.0, tau["eta_over_s"], tau["T_R_GeV"],
                           tau["n_unit_fm3"], tau["dx_fm"], landau_tol, landau_maxit, LANDAU[landau])
    return LatticeDesc(nx, ny, BC[bc[0]], BC[bc[1]], TAU_CONST, float(tau), 0, 0, 0, 0, landau_tol, landau_maxit,
                       LANDAU[landau])


def check_lattice(bases, zeta, v0, nx, ny, dim=2, precision="fp64", **lattice):
    """Host-only check of a lattice description (no GPU): raises RlbmError
    with the library's reason when rlbm_init_fields would reject it."""
    d = make_desc(bases, zeta, v0, dim, precision)
    lat = lattice_desc(nx, ny, **lattice)
    _check(lib().rlbm_check_lattice(ctypes.byref(d), ctypes.byref(lat)))


def info_dict(info, ngroups=6):
    return {"q3": info.q3, "q": info.q, "v0": info.v0, "v0_lo": info.v0_lo, "v0_hi": info.v0_hi,
            "weights": [info.weights[i] for i in range(ngroups)], "ortho_residual": info.ortho_residual,
            "max_shift": info.max_shift, "cond": info.cond}


def solve_stencil(bases, zeta, v0=0.0, dim=2, v0_lo=0.0, v0_hi=0.0, order=2, weights=None):
    """Host-only stencil construction (no GPU): dict of the stencil info
    (order 2: six groups; order 3: eleven)."""
    d = make_desc(bases, zeta, v0, dim, "fp64", v0_lo=v0_lo, v0_hi=v0_hi, order=order, weights=weights)
    info = StencilInfo()
    _check(lib().rlbm_solve_stencil(ctypes.byref(d), ctypes.byref(info)))
    return info_dict(info, len(bases))


def class_table(bases, zeta, v0, dim=2):
    """Host-only population-class table: (disp [q,2], mom [q,3], M [q,10]) as lists."""
    import numpy as np
    d = make_desc(bases, zeta, v0, dim)
    cap = 160
    disp = (ctypes.c_int * (2 * cap))()
    mom = (ctypes.c_double * (3 * cap))()
    M = (ctypes.c_double * (10 * cap))()
    _check(lib().rlbm_class_table(ctypes.byref(d), cap, disp, mom, M))
    q = solve_stencil(bases, zeta, v0, dim)["q"]
    return (np.array(disp[:2 * q]).reshape(q, 2), np.array(mom[:3 * q]).reshape(q, 3),
            np.array(M[:10 * q]).reshape(q, 10))


def eos_temperature_host(zeta, e):
    """Host evaluation of the library's inverse-EOS table (no GPU)."""
    import numpy as np
    e = np.ascontiguousarray(e, dtype=np.float64)
    T = np.empty_like(e)
    dp = ctypes.POINTER(ctypes.c_double)
    _check(lib().rlbm_eos_temperature_host(float(zeta), e.ctypes.data_as(dp), e.size, T.ctypes.data_as(dp)))
    return T


MLP_NPARAM = 9155


class MLP:
    """The learned Landau-frame guess network on the current device.
    params: 9155 float32 values (W1, b1, W2, b2, W3, b3, W4, b4); norm: 24
    float32 values mx[9], sx[9], my[3], sy[3]."""

    def __init__(self, params, norm, max_batch=8192):
        import numpy as np
        import torch
        self.torch = torch
        p = np.ascontiguousarray(params, dtype=np.float32)
        nrm = np.ascontiguousarray(norm, dtype=np.float32)
        assert p.size == MLP_NPARAM and nrm.size == 24
        fp = ctypes.POINTER(ctypes.c_float)
        h = ctypes.c_void_p()
        _check(lib().rlbm_mlp_create(ctypes.byref(h), p.ctypes.data_as(fp), nrm.ctypes.data_as(fp), int(max_batch)))
        self.h = h
        self.max_batch = max_batch

    def __del__(self):
        try:
            if getattr(self, "h", None):
                lib().rlbm_mlp_destroy(self.h)
                self.h = None
        except Exception:
            pass

    def _stream(self):
        return ctypes.c_void_p(self.torch.cuda.current_stream().cuda_stream)

    def train_step(self, raw9, target, lr):
        """raw9 [B, 9], target [B, 3] (eps, ux, uy): CUDA float32; returns the loss."""
        assert raw9.dtype == self.torch.float32 and target.dtype == self.torch.float32
        loss = ctypes.c_float()
        _check(lib().rlbm_mlp_train_step(self.h, raw9.data_ptr(), target.data_ptr(), raw9.shape[0], float(lr),
                                         ctypes.byref(loss), self._stream()))
        return loss.value

    def predict(self, raw9):
        out = self.torch.empty((raw9.shape[0], 3), dtype=self.torch.float32, device=raw9.device)
        _check(lib().rlbm_mlp_predict(self.h, raw9.data_ptr(), raw9.shape[0], out.data_ptr(), self._stream()))
        return out

    def params(self):
        import numpy as np
        p = np.empty(MLP_NPARAM, dtype=np.float32)
        g = np.empty(MLP_NPARAM, dtype=np.float32)
        fp = ctypes.POINTER(ctypes.c_float)
        _check(lib().rlbm_mlp_get_params(self.h, p.ctypes.data_as(fp), g.ctypes.data_as(fp)))
        return p, g


class Solver:
    """One lattice on the current CUDA (HIP) device.

    bases: group base vectors; zeta = m/T_R; v0 (<= 0: search the positive
    window); precision 'fp64' | 'fp32' | 'fp16' (deviation storage)."""

    def __init__(self, bases, zeta, v0, dim=2, precision="fp64", n_ref=1.0, T_ref=1.0, v0_lo=0.0, v0_hi=0.0,
                 order=2, weights=None):
        import torch
        self.torch = torch
        self.precision = precision
        self.dim = dim
        self.order = order
        self._desc = make_desc(bases, zeta, v0, dim, precision, n_ref, T_ref, v0_lo, v0_hi, order, weights)
        info = StencilInfo()
        ctx = ctypes.c_void_p()
        _check(lib().rlbm_init_stencil(ctypes.byref(ctx), ctypes.byref(self._desc), ctypes.byref(info)))
        self.ctx = ctx
        self.info = info_dict(info, len(bases))
        self.nx = self.ny = None
        self.pop = None

    def __del__(self):
        try:
            if getattr(self, "ctx", None):
                lib().rlbm_destroy(self.ctx)
                self.ctx = None
        except Exception:
            pass

    def _stream(self):
        return ctypes.c_void_p(self.torch.cuda.current_stream().cuda_stream)

    def population_bytes(self, nx, ny):
        return lib().rlbm_population_bytes(self.ctx, nx, ny)

    def init_fields(self, n, T, ux, uy, bc=("periodic", "periodic"), tau=1.0, landau_tol=0.0, landau_maxit=0,
                    landau="newton", noalloc=False):
        """n, T, ux, uy: CUDA float64 tensors [ny, nx].  tau: float, or dict with
        eta_over_s, T_R_GeV, n_unit_fm3, dx_fm for the eta/s rule.  noalloc:
        use rlbm_init_fields_noalloc (health slots in the library's static
        device array)."""
        torch = self.torch
        ny, nx = n.shape
        for a in (n, T, ux, uy):
            assert a.is_cuda and a.dtype == torch.float64 and a.is_contiguous() and tuple(a.shape) == (ny, nx)
        lat = lattice_desc(nx, ny, bc, tau, landau_tol, landau_maxit, landau)
        nbytes = self.population_bytes(nx, ny)
        self.pop = [torch.empty(nbytes, dtype=torch.uint8, device=n.device) for _ in range(2)]
        self._fields = (n, T, ux, uy)
        fn = lib().rlbm_init_fields_noalloc if noalloc else lib().rlbm_init_fields
        _check(fn(self.ctx, ctypes.byref(lat), n.data_ptr(), T.data_ptr(), ux.data_ptr(), uy.data_ptr(),
                  self.pop[0].data_ptr(), self.pop[1].data_ptr(), nbytes, self._stream()), self.ctx)
        self.nx, self.ny = nx, ny

    def step(self, nsteps=1):
        _check(lib().rlbm_step(self.ctx, int(nsteps), self._stream()), self.ctx)

    def moments(self, raw=False):
        """Fields of the current pre-collision state as CUDA float64 tensors."""
        torch = self.torch
        dev = self.pop[0].device
        out = {k: torch.empty((self.ny, self.nx), dtype=torch.float64, device=dev)
               for k in ("n", "eps", "T", "P", "ux", "uy")}
        raw9 = torch.empty((9, self.ny, self.nx), dtype=torch.float64, device=dev) if raw else None
        _check(lib().rlbm_moments(self.ctx, out["n"].data_ptr(), out["eps"].data_ptr(), out["T"].data_ptr(),
                                  out["P"].data_ptr(), out["ux"].data_ptr(), out["uy"].data_ptr(),
                                  raw9.data_ptr() if raw else None, self._stream()), self.ctx)
        if raw:
            out["raw9"] = raw9
        return out

    def health(self, reset=False):
        f = ctypes.c_uint()
        s = ctypes.c_ulonglong()
        m = ctypes.c_uint()
        rc = lib().rlbm_get_health(self.ctx, ctypes.byref(f), ctypes.byref(s), ctypes.byref(m), int(reset),
                                   self._stream())
        if rc not in (RLBM_OK, RLBM_ENUMERIC):
            _check(rc, self.ctx)
        return {"flags": f.value, "iter_sum": s.value, "iter_max": m.value, "fatal": rc == RLBM_ENUMERIC}

    def set_landau_guess(self, mlp):
        """Start every Landau solve from the network's guess (None: plain start)."""
        self._mlp = mlp
        _check(lib().rlbm_set_landau_guess(self.ctx, mlp.h if mlp is not None else None), self.ctx)

    def set_warm_start(self, enable=True):
        """Start every Landau solve from the frame each site converged to in
        the previous step (exclusive with the learned guess)."""
        _check(lib().rlbm_set_warm_start(self.ctx, int(bool(enable))), self.ctx)

    def landau_guess_fields(self):
        torch = self.torch
        out = torch.empty((3, self.ny, self.nx), dtype=torch.float32, device=self.pop[0].device)
        _check(lib().rlbm_landau_guess_fields(self.ctx, out.data_ptr(), self._stream()), self.ctx)
        return out

    def step_count(self):
        return lib().rlbm_step_count(self.ctx)

    def set_step_variant(self, variant):
        """"auto" (the generated fixed-stencil kernel when one matches this
        stencil) or "table" (always the table-driven kernel)."""
        _check(lib().rlbm_set_step_variant(self.ctx, {"auto": STEP_AUTO, "table": STEP_TABLE}[variant]), self.ctx)

    def step_kernel(self):
        """Which kernel the next step runs: "table" or "fixed"."""
        return {STEP_TABLE: "table", STEP_FIXED: "fixed"}[lib().rlbm_step_kernel(self.ctx)]

    def save_state(self):
        torch = self.torch
        buf = torch.empty_like(self.pop[0])
        step = ctypes.c_longlong()
        flag = ctypes.c_int()
        _check(lib().rlbm_save_state(self.ctx, buf.data_ptr(), buf.numel(), ctypes.byref(step), ctypes.byref(flag),
                                     self._stream()), self.ctx)
        return buf, step.value, flag.value

    def load_state(self, buf, step, flag):
        _check(lib().rlbm_load_state(self.ctx, buf.data_ptr(), buf.numel(), int(step), int(flag), self._stream()),
               self.ctx)

    def populations(self):
        """Current state buffer as a flat tensor in storage dtype: rows of the
        lattice (with ghost rows), each holding the q class rows of W elements
        back to back."""
        import numpy as np
        torch = self.torch
        dt = {"fp64": torch.float64, "fp32": torch.float32, "fp16": torch.float16}[self.precision]
        buf = self.pop[0] if (self.step_count() % 2 == 0) else self.pop[1]
        return buf.view(dt)


def device_copy(dst, src, workgroups=2048):
    """Streaming copy of src into dst (CUDA tensors of equal byte size, a
    multiple of 16) on the current stream."""
    import torch
    nbytes = src.numel() * src.element_size()
    assert dst.numel() * dst.element_size() == nbytes
    _check(lib().rlbm_device_copy(dst.data_ptr(), src.data_ptr(), nbytes, int(workgroups),
                                  ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)))


class Solver3D(Solver):
    """A lattice on the 3D layout on the current device; fields are CUDA
    float64 tensors [nz, ny, nx].  Second order: dim 3 (Nx x Ny x Nz, every
    population of the stencil).  Third order (order=3, eleven groups, float64):
    dim 3, or dim 2 / 1 with merged classes on an Nx x Ny x 1 / Nx x 1 x 1
    lattice."""

    def __init__(self, bases, zeta, v0, precision="fp64", n_ref=1.0, T_ref=1.0, v0_lo=0.0, v0_hi=0.0,
                 order=2, dim=3, weights=None):
        super().__init__(bases, zeta, v0, dim=dim, precision=precision, n_ref=n_ref, T_ref=T_ref, v0_lo=v0_lo,
                         v0_hi=v0_hi, order=order, weights=weights)
        self.nz = None

    def population_bytes3(self, nx, ny, nz):
        return lib().rlbm_population_bytes3(self.ctx, nx, ny, nz)

    def init_fields(self, n, T, ux, uy, uz, bc=("periodic", "periodic", "periodic"), tau=1.0, landau_tol=0.0,
                    landau_maxit=0):
        torch = self.torch
        nz, ny, nx = n.shape
        for a in (n, T, ux, uy, uz):
            assert a.is_cuda and a.dtype == torch.float64 and a.is_contiguous() and tuple(a.shape) == (nz, ny, nx)
        lat = lattice_desc(nx, ny, bc[:2], tau, landau_tol, landau_maxit, "newton")
        lat.nz = nz
        lat.bc_z = BC[bc[2]]
        nbytes = self.population_bytes3(nx, ny, nz)
        self.pop = [torch.empty(nbytes, dtype=torch.uint8, device=n.device) for _ in range(2)]
        self._fields = (n, T, ux, uy, uz)
        _check(lib().rlbm_init_fields3(self.ctx, ctypes.byref(lat), n.data_ptr(), T.data_ptr(), ux.data_ptr(),
                                       uy.data_ptr(), uz.data_ptr(), self.pop[0].data_ptr(), self.pop[1].data_ptr(),
                                       nbytes, self._stream()), self.ctx)
        self.nx, self.ny, self.nz = nx, ny, nz

    def moments(self, raw=False):
        torch = self.torch
        dev = self.pop[0].device
        shp = (self.nz, self.ny, self.nx)
        out = {k: torch.empty(shp, dtype=torch.float64, device=dev) for k in ("n", "eps", "T", "P", "ux", "uy", "uz")}
        raw14 = torch.empty((14,) + shp, dtype=torch.float64, device=dev) if raw else None
        _check(lib().rlbm_moments3(self.ctx, out["n"].data_ptr(), out["eps"].data_ptr(), out["T"].data_ptr(),
                                   out["P"].data_ptr(), out["ux"].data_ptr(), out["uy"].data_ptr(),
                                   out["uz"].data_ptr(), raw14.data_ptr() if raw else None, self._stream()), self.ctx)
        if raw:
            out["raw14"] = raw14
        return out


class Batch:
    """Batched 1D problems advanced in one persistent launch.  stencils: list of
    Solver objects built with dim=1, precision='fp32'; problems: list of dicts
    with nx, stencil (index), eta_over_s, T_R_GeV, n_unit_fm3, dx_fm."""

    def __init__(self, stencils, problems, landau_tol=0.0, landau_maxit=0):
        import torch
        self.torch = torch
        self._stencils = stencils
        arr = (ctypes.c_void_p * len(stencils))(*[s.ctx.value for s in stencils])
        pr = (Problem * len(problems))(*[Problem(p["nx"], p["stencil"], p["eta_over_s"], p["T_R_GeV"],
                                                 p["n_unit_fm3"], p["dx_fm"]) for p in problems])
        h = ctypes.c_void_p()
        _check(lib().rlbm_batch_create(ctypes.byref(h), len(stencils), arr, len(problems), pr, float(landau_tol),
                                       int(landau_maxit)))
        self.h = h
        self.sites = lib().rlbm_batch_sites(h)
        self.problems = problems

    def __del__(self):
        try:
            if getattr(self, "h", None):
                lib().rlbm_batch_destroy(self.h)
                self.h = None
        except Exception:
            pass

    def _stream(self):
        return ctypes.c_void_p(self.torch.cuda.current_stream().cuda_stream)

    def init(self, n, T, ux):
        torch = self.torch
        nbytes = lib().rlbm_batch_population_bytes(self.h)
        self.pop = [torch.empty(nbytes, dtype=torch.uint8, device=n.device) for _ in range(2)]
        self._fields = (n, T, ux)
        _check(lib().rlbm_batch_init(self.h, n.data_ptr(), T.data_ptr(), ux.data_ptr(), self.pop[0].data_ptr(),
                                     self.pop[1].data_ptr(), nbytes, self._stream()))

    def step(self, nsteps, sample_every=0):
        """Advances nsteps in one launch; returns the samples tensor
        [ceil(nsteps / sample_every), sites, 12] when sample_every > 0."""
        torch = self.torch
        samples = None
        if sample_every > 0:
            ns = (nsteps + sample_every - 1) // sample_every
            samples = torch.empty((ns, self.sites, 12), dtype=torch.float32, device=self.pop[0].device)
        _check(lib().rlbm_batch_step_persistent(self.h, int(nsteps), int(sample_every),
                                                samples.data_ptr() if samples is not None else None,
                                                self._stream()))
        return samples

    def moments(self):
        torch = self.torch
        out = {k: torch.empty(self.sites, dtype=torch.float64, device=self.pop[0].device)
               for k in ("n", "eps", "T", "P", "ux")}
        _check(lib().rlbm_batch_moments(self.h, out["n"].data_ptr(), out["eps"].data_ptr(), out["T"].data_ptr(),
                                        out["P"].data_ptr(), out["ux"].data_ptr(), self._stream()))
        return out

    def occupancy(self):
        """Cooperative grid of the step: workgroups launched, resident limit, tiles."""
        w, r, t = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        _check(lib().rlbm_batch_occupancy(self.h, ctypes.byref(w), ctypes.byref(r), ctypes.byref(t)))
        return {"workgroups": w.value, "resident_limit": r.value, "tiles": t.value}

    def health(self):
        f = ctypes.c_uint()
        s = ctypes.c_ulonglong()
        m = ctypes.c_uint()
        rc = lib().rlbm_batch_get_health(self.h, ctypes.byref(f), ctypes.byref(s), ctypes.byref(m), self._stream())
        if rc not in (RLBM_OK, RLBM_ENUMERIC):
            _check(rc)
        return {"flags": f.value, "iter_sum": s.value, "iter_max": m.value, "fatal": rc == RLBM_ENUMERIC}
