"""Thin Python binding of the ASDSM C ABI (``include/asdsm.h``, ``include/asdsm_learn.h``).

Argument marshalling only: every step of the method runs inside ``libasdsm.so`` on the GPU.  PyTorch
provides the device memory (float64 tensors, the byte workspace) and the stream.  There is no CPU
fallback: if the library is missing or no GPU is present, the calls raise.
"""
from __future__ import annotations

import ctypes
from ctypes import POINTER, byref, c_double, c_int, c_int64, c_size_t, c_uint, c_uint64, c_void_p
from pathlib import Path

LIB_PATH = Path(__file__).resolve().with_name("libasdsm.so")

ASDSM_OK, ASDSM_STAGNATED, ASDSM_MAXITER = 0, 1, 2
ASDSM_E_ARG, ASDSM_E_NESTING, ASDSM_E_WORKSPACE = -1, -2, -3
ASDSM_E_NUMERIC, ASDSM_E_DEVICE, ASDSM_E_UNSUPPORTED = -4, -5, -6
NPHASE = 8
PHASES = ("rhs", "transform", "line", "skeleton", "filler", "dots", "update", "learned")
STATUS_NAMES = {0: "ok", 1: "stagnated", 2: "maxiter"}
PRECISIONS = {"fp64": 0, "fp32": 1}  # asdsm_opts.precision: FP64 or FP32 error-phase submesh solves

# symbols declared in include/asdsm.h
# transform tile shapes of the anisotropic solves (ASDSM_TILE_* in include/asdsm.h)
TILES = {"auto": 0, "32x32": 1, "64x32": 2, "32x64": 3, "64x64": 4, "plane": 5}
EXPORTED = ("asdsm_plan", "asdsm_workspace_size", "asdsm_set_workspace", "asdsm_solve",
            "asdsm_residual", "asdsm_mesh_solve", "asdsm_destroy", "asdsm_last_error",
            "asdsm_batch_create", "asdsm_batch_solve", "asdsm_batch_destroy", "asdsm_autotune",
            "asdsm_tile_name", "asdsm_set_tile", "asdsm_get_tile", "asdsm_probe_mfma_scratch_bytes",
            "asdsm_probe_mfma_f64", "asdsm_probe_copy", "asdsm_profile_count", "asdsm_profile_entry", "asdsm_line_axes",
            "asdsm_residual_noalloc")
# symbols declared in include/asdsm_learn.h
EXPORTED_LEARN = ("asdsm_net_create", "asdsm_net_param_count", "asdsm_net_workspace_size",
                  "asdsm_net_set_workspace", "asdsm_net_params", "asdsm_net_forward",
                  "asdsm_net_gradient", "asdsm_net_bind", "asdsm_net_features",
                  "asdsm_solve_learned", "asdsm_net_adam", "asdsm_net_destroy")
NET_LOSSES = {"mse": 0, "residual": 1}  # asdsm_net_gradient loss kinds


class AsdsmError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"ASDSM error {code}: {msg}")
        self.code = code


class Opts(ctypes.Structure):
    _fields_ = [("max_iter", c_int), ("rtol", c_double), ("stag_window", c_int),
                ("stag_eta", c_double), ("resume", c_int), ("k0", c_int64),
                ("hist", POINTER(c_double)), ("step_hist", POINTER(c_double)), ("profile", c_int),
                ("eager", c_int), ("precision", c_int), ("skeleton", c_int)]


class Stats(ctypes.Structure):
    _fields_ = [("status", c_int), ("iterations", c_int), ("bnorm", c_double),
                ("r0norm", c_double), ("rnorm", c_double), ("phase_ms", c_double * NPHASE),
                ("phase_launches", c_int * NPHASE), ("phase_flops", c_double * NPHASE),
                ("phase_bytes", c_double * NPHASE), ("total_ms", c_double), ("precision", c_int)]


_lib = None


def load_library():
    """Load libasdsm.so (built in-tree); raise if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not LIB_PATH.exists():
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_2303_01163_amd.build`")
    lib = ctypes.CDLL(str(LIB_PATH))
    lib.asdsm_plan.argtypes = [POINTER(c_void_p), c_int, POINTER(c_double), POINTER(c_double),
                               c_int, c_int, c_uint64, c_void_p]
    lib.asdsm_plan.restype = c_int
    lib.asdsm_workspace_size.argtypes = [c_void_p, POINTER(c_size_t)]
    lib.asdsm_workspace_size.restype = c_int
    lib.asdsm_set_workspace.argtypes = [c_void_p, c_void_p, c_size_t]
    lib.asdsm_set_workspace.restype = c_int
    lib.asdsm_solve.argtypes = [c_void_p, c_void_p, c_void_p, c_void_p, POINTER(Opts), POINTER(Stats)]
    lib.asdsm_solve.restype = c_int
    lib.asdsm_residual.argtypes = [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, POINTER(c_double)]
    lib.asdsm_residual.restype = c_int
    lib.asdsm_mesh_solve.argtypes = [c_void_p, c_uint, c_void_p, c_void_p]
    lib.asdsm_mesh_solve.restype = c_int
    lib.asdsm_destroy.argtypes = [c_void_p]
    lib.asdsm_destroy.restype = None
    lib.asdsm_autotune.argtypes = [c_void_p, c_int, POINTER(c_int), POINTER(c_double)]
    lib.asdsm_autotune.restype = c_int
    lib.asdsm_tile_name.argtypes = [c_int]
    lib.asdsm_tile_name.restype = ctypes.c_char_p
    lib.asdsm_set_tile.argtypes = [c_void_p, c_int]
    lib.asdsm_set_tile.restype = c_int
    lib.asdsm_get_tile.argtypes = [c_void_p, POINTER(c_int)]
    lib.asdsm_get_tile.restype = c_int
    lib.asdsm_probe_mfma_scratch_bytes.argtypes = []
    lib.asdsm_probe_mfma_scratch_bytes.restype = c_size_t
    lib.asdsm_probe_mfma_f64.argtypes = [c_void_p, c_int, c_void_p, POINTER(c_double)]
    lib.asdsm_probe_mfma_f64.restype = c_int
    lib.asdsm_probe_copy.argtypes = [c_void_p, c_void_p, c_size_t, c_int, c_void_p, POINTER(c_double)]
    lib.asdsm_probe_copy.restype = c_int
    lib.asdsm_residual_noalloc.argtypes = [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, POINTER(c_double)]
    lib.asdsm_residual_noalloc.restype = c_int
    lib.asdsm_line_axes.argtypes = [c_void_p, POINTER(c_int), POINTER(c_int)]
    lib.asdsm_line_axes.restype = c_int
    lib.asdsm_profile_count.argtypes = [c_void_p]
    lib.asdsm_profile_count.restype = c_int
    lib.asdsm_profile_entry.argtypes = [c_void_p, c_int, ctypes.c_char_p, c_int, POINTER(c_int),
                                        POINTER(c_double), POINTER(c_int), POINTER(c_int),
                                        POINTER(c_double), POINTER(c_double)]
    lib.asdsm_profile_entry.restype = c_int
    lib.asdsm_batch_create.argtypes = [POINTER(c_void_p), POINTER(c_void_p), c_int]
    lib.asdsm_batch_create.restype = c_int
    lib.asdsm_batch_solve.argtypes = [c_void_p, POINTER(c_void_p), POINTER(c_void_p), POINTER(c_void_p),
                                      POINTER(Opts), POINTER(Stats)]
    lib.asdsm_batch_solve.restype = c_int
    lib.asdsm_batch_destroy.argtypes = [c_void_p]
    lib.asdsm_batch_destroy.restype = None
    F = POINTER(ctypes.c_float)
    lib.asdsm_net_create.argtypes = [POINTER(c_void_p), c_int, c_uint64, c_void_p]
    lib.asdsm_net_create.restype = c_int
    lib.asdsm_net_param_count.argtypes = [c_void_p, POINTER(c_size_t)]
    lib.asdsm_net_param_count.restype = c_int
    lib.asdsm_net_workspace_size.argtypes = [c_void_p, POINTER(c_size_t)]
    lib.asdsm_net_workspace_size.restype = c_int
    lib.asdsm_net_set_workspace.argtypes = [c_void_p, c_void_p, c_size_t]
    lib.asdsm_net_set_workspace.restype = c_int
    lib.asdsm_net_params.argtypes = [c_void_p, F, c_int]
    lib.asdsm_net_params.restype = c_int
    lib.asdsm_net_forward.argtypes = [c_void_p, c_void_p, c_void_p]
    lib.asdsm_net_forward.restype = c_int
    lib.asdsm_net_gradient.argtypes = [c_void_p, c_void_p, c_void_p, c_int, POINTER(c_double), F]
    lib.asdsm_net_gradient.restype = c_int
    lib.asdsm_net_bind.argtypes = [c_void_p, c_void_p]
    lib.asdsm_net_bind.restype = c_int
    lib.asdsm_net_features.argtypes = [c_void_p, c_void_p, c_double, POINTER(c_int), c_void_p, c_void_p]
    lib.asdsm_net_features.restype = c_int
    lib.asdsm_solve_learned.argtypes = [c_void_p, c_void_p, c_double, c_void_p, c_void_p, c_void_p,
                                        POINTER(Opts), POINTER(Stats), POINTER(c_int)]
    lib.asdsm_solve_learned.restype = c_int
    lib.asdsm_net_adam.argtypes = [c_void_p, ctypes.c_float]
    lib.asdsm_net_adam.restype = c_int
    lib.asdsm_net_destroy.argtypes = [c_void_p]
    lib.asdsm_net_destroy.restype = None
    lib.asdsm_last_error.argtypes = []
    lib.asdsm_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _check(rc: int) -> int:
    if rc < 0:
        raise AsdsmError(rc, load_library().asdsm_last_error().decode())
    return rc


def _dptr(t, n=None, name="tensor"):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA tensor")
    if t.dtype != torch.float64 or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous float64 tensor")
    if n is not None and t.numel() != n:
        raise ValueError(f"{name} has {t.numel()} elements, expected {n}")
    return c_void_p(t.data_ptr())


def _fptr(t, n=None, name="tensor"):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA tensor")
    if t.dtype != torch.float32 or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous float32 tensor")
    if n is not None and t.numel() != n:
        raise ValueError(f"{name} has {t.numel()} elements, expected {n}")
    return c_void_p(t.data_ptr())


def _opts(max_iter, rtol, stag_window, stag_eta, resume, k0, profile, eager, precision, skeleton=False):
    hist = (c_double * (max_iter + 1))()
    steps = (c_double * max(max_iter, 1))()
    o = Opts(max_iter=int(max_iter), rtol=float(rtol), stag_window=int(stag_window),
             stag_eta=float(stag_eta), resume=1 if resume else 0, k0=int(k0),
             hist=ctypes.cast(hist, POINTER(c_double)),
             step_hist=ctypes.cast(steps, POINTER(c_double)), profile=1 if profile else 0,
             eager=1 if eager else 0, precision=PRECISIONS[precision], skeleton=1 if skeleton else 0)
    return o, hist, steps


def _info(rc, st, hist, steps, profile):
    it = st.iterations
    info = {
        "status": st.status if rc >= 0 else rc, "status_name": STATUS_NAMES.get(st.status, str(st.status)),
        "iterations": it, "bnorm": st.bnorm, "r0norm": st.r0norm, "rnorm": st.rnorm,
        "res_hist": [hist[i] for i in range(it + 1)] if hist is not None else None,
        "step_hist": [steps[i] for i in range(it)] if steps is not None else None,
        "precision": {v: k for k, v in PRECISIONS.items()}[st.precision],
    }
    if profile:
        info["phase_ms"] = {PHASES[q]: st.phase_ms[q] for q in range(NPHASE)}
        info["phase_launches"] = {PHASES[q]: st.phase_launches[q] for q in range(NPHASE)}
        info["phase_flops"] = {PHASES[q]: st.phase_flops[q] for q in range(NPHASE)}
        info["phase_bytes"] = {PHASES[q]: st.phase_bytes[q] for q in range(NPHASE)}
        info["total_ms"] = st.total_ms
    return info


class Plan:
    """An ASDSM plan on one GPU: d in {2,3,4}, per-axis alpha/beta, fine level L, coarse level L_c."""

    def __init__(self, d, alpha, beta, level, coarse_level=0, seed=0, device=None, stream=None):
        import torch
        lib = load_library()
        if not torch.cuda.is_available():
            raise RuntimeError("ASDSM needs a HIP GPU; none is available")
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.d = int(d)
        self.level = int(level)
        self.coarse_level = int(coarse_level) if coarse_level else self.level // 2
        self.n_f = 2 ** self.level - 1
        self.n_c = 2 ** self.coarse_level - 1
        self.seed = int(seed)
        a = (c_double * self.d)(*[float(x) for x in alpha])
        b = (c_double * self.d)(*[float(x) for x in beta])
        self._h = c_void_p()
        with torch.cuda.device(self.device):
            _check(lib.asdsm_plan(byref(self._h), self.d, a, b, self.level, self.coarse_level,
                                  c_uint64(self.seed & 0xFFFFFFFFFFFFFFFF),
                                  c_void_p(self.stream.cuda_stream)))
            nbytes = c_size_t()
            _check(lib.asdsm_workspace_size(self._h, byref(nbytes)))
            self.workspace_bytes = int(nbytes.value)
            self._ws = torch.empty(self.workspace_bytes + 256, dtype=torch.uint8, device=self.device)
            base = self._ws.data_ptr()
            aligned = (base + 255) // 256 * 256
            _check(lib.asdsm_set_workspace(self._h, c_void_p(aligned), c_size_t(self.workspace_bytes)))

    def attach_workspace(self):
        """Allocate a fresh device workspace and attach it (asdsm_set_workspace); returns the
        previous workspace tensor, which the plan no longer uses."""
        import torch
        old = self._ws
        with torch.cuda.device(self.device):
            self._ws = torch.empty(self.workspace_bytes + 256, dtype=torch.uint8, device=self.device)
            aligned = (self._ws.data_ptr() + 255) // 256 * 256
            _check(load_library().asdsm_set_workspace(self._h, c_void_p(aligned), c_size_t(self.workspace_bytes)))
        return old

    @property
    def n_fine(self) -> int:
        return self.n_f ** self.d

    def mesh_shape(self, mask: int) -> tuple:
        """Canonical layout of mesh M_S: fine axes (increasing) then coarse axes, first fastest."""
        fine = [j for j in range(self.d) if not (mask >> j) & 1]
        coarse = [j for j in range(self.d) if (mask >> j) & 1]
        return tuple([self.n_f] * len(fine) + [self.n_c] * len(coarse)), fine + coarse

    @property
    def n_faces(self) -> int:
        return 2 * self.d * self.n_f ** (self.d - 1)

    def solve(self, s, g, u=None, max_iter=50, rtol=1e-10, stag_window=3, stag_eta=1e-3,
              resume=False, k0=0, profile=False, eager=False, precision="fp64", skeleton=False):
        import torch
        lib = load_library()
        if u is None:
            u = torch.empty(self.n_fine, dtype=torch.float64, device=self.device)
        o, hist, steps = _opts(max_iter, rtol, stag_window, stag_eta, resume, k0, profile, eager, precision,
                               skeleton)
        st = Stats()
        with torch.cuda.device(self.device):
            rc = _check(lib.asdsm_solve(self._h, _dptr(s, self.n_fine, "s"), _dptr(g, self.n_faces, "g"),
                                        _dptr(u, self.n_fine, "u"), byref(o), byref(st)))
        return u, _info(rc, st, hist, steps, profile)

    def set_tile(self, tile):
        """Force the transform tile shape (asdsm_set_tile): a TILES key or its integer code."""
        code = TILES[tile] if isinstance(tile, str) else int(tile)
        _check(load_library().asdsm_set_tile(self._h, code))

    def tile_name(self):
        """Name of the tile shape the anisotropic solves use now (asdsm_get_tile)."""
        lib = load_library()
        t = c_int()
        _check(lib.asdsm_get_tile(self._h, byref(t)))
        return lib.asdsm_tile_name(t.value).decode()

    def autotune(self, repeats=10):
        """Choose this plan's FP64 transform tile shape by timing (asdsm_autotune)."""
        import torch
        lib = load_library()
        tile, ms = c_int(), c_double()
        with torch.cuda.device(self.device):
            _check(lib.asdsm_autotune(self._h, int(repeats), byref(tile), byref(ms)))
        return {"tile": lib.asdsm_tile_name(tile.value).decode(), "ms_per_aniso_solve": ms.value}

    def line_axes(self):
        """{mesh mask: (line axis or -1, refinement sweeps)} for every submesh (asdsm_line_axes)."""
        lib = load_library()
        n = 1 << self.d
        ax, sw = (c_int * n)(), (c_int * n)()
        _check(lib.asdsm_line_axes(self._h, ax, sw))
        return {m: (ax[m], sw[m]) for m in range(1, n)}

    def kernel_profile(self):
        """Launch groups of the last profiled solve by kind (asdsm_profile_count/entry): a list of
        dicts with name, phase, ms, groups, launches, flops, bytes."""
        lib = load_library()
        n = _check(lib.asdsm_profile_count(self._h))
        out = []
        for i in range(n):
            name = ctypes.create_string_buffer(96)
            ph, gr, la = c_int(), c_int(), c_int()
            ms, fl, by = c_double(), c_double(), c_double()
            _check(lib.asdsm_profile_entry(self._h, i, name, 96, byref(ph), byref(ms), byref(gr),
                                           byref(la), byref(fl), byref(by)))
            out.append({"name": name.value.decode(), "phase": PHASES[ph.value], "ms": ms.value,
                        "groups": gr.value, "launches": la.value, "flops": fl.value, "bytes": by.value})
        return out

    def residual(self, u, s, g, want_r=True):
        import torch
        lib = load_library()
        r = torch.empty(self.n_fine, dtype=torch.float64, device=self.device) if want_r else None
        nrm = c_double()
        with torch.cuda.device(self.device):
            _check(lib.asdsm_residual(self._h, _dptr(u, self.n_fine, "u"), _dptr(s, self.n_fine, "s"),
                                      _dptr(g, 2 * self.d * self.n_f ** (self.d - 1), "g"),
                                      _dptr(r, self.n_fine, "r") if want_r else None, byref(nrm)))
        return r, nrm.value

    def residual_noalloc(self, u, s, g, r=None):
        """r = b - A u and ||r||_2 through the allocation-free entry point (asdsm_residual_noalloc):
        r, if given, is a caller-owned device tensor of N_f^d doubles; returns (r, ||r||_2)."""
        import torch
        lib = load_library()
        nrm = c_double()
        with torch.cuda.device(self.device):
            _check(lib.asdsm_residual_noalloc(self._h, _dptr(u, self.n_fine, "u"), _dptr(s, self.n_fine, "s"),
                                              _dptr(g, 2 * self.d * self.n_f ** (self.d - 1), "g"),
                                              _dptr(r, self.n_fine, "r") if r is not None else None,
                                              byref(nrm)))
        return r, nrm.value

    def mesh_solve(self, mask: int, rhs):
        import torch
        lib = load_library()
        shape, _ = self.mesh_shape(mask)
        n = 1
        for e in shape:
            n *= e
        x = torch.empty(n, dtype=torch.float64, device=self.device)
        with torch.cuda.device(self.device):
            _check(lib.asdsm_mesh_solve(self._h, c_uint(mask), _dptr(rhs, n, "rhs"), _dptr(x, n, "x")))
        return x

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load_library().asdsm_destroy(self._h)
            self._h = c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Independent problems solved together (asdsm_batch_*): one graph replay advances every
    member by two refinement steps.  The plans are borrowed and must outlive the batch."""

    def __init__(self, plans):
        import torch
        lib = load_library()
        self.plans = list(plans)
        arr = (c_void_p * len(self.plans))(*[p._h.value for p in self.plans])
        self._h = c_void_p()
        with torch.cuda.device(self.plans[0].device):
            _check(lib.asdsm_batch_create(byref(self._h), arr, len(self.plans)))

    def solve(self, ss, gs, us=None, max_iter=50, rtol=1e-10, stag_window=3, stag_eta=1e-3,
              precision="fp64", profile=False, eager=False, skeleton=False):
        """Returns (list of u, list of info); the histories are not collected in a batch.  With
        skeleton=True the d = 3 members run the skeleton-sparse loop."""
        import torch
        lib = load_library()
        n = len(self.plans)
        if us is None:
            us = [torch.empty(p.n_fine, dtype=torch.float64, device=p.device) for p in self.plans]
        sp = (c_void_p * n)(*[_dptr(ss[i], self.plans[i].n_fine, "s").value for i in range(n)])
        gp = (c_void_p * n)(*[_dptr(gs[i], self.plans[i].n_faces, "g").value for i in range(n)])
        up = (c_void_p * n)(*[_dptr(us[i], self.plans[i].n_fine, "u").value for i in range(n)])
        o = Opts(max_iter=int(max_iter), rtol=float(rtol), stag_window=int(stag_window),
                 stag_eta=float(stag_eta), resume=0, k0=0, hist=None, step_hist=None,
                 profile=1 if profile else 0, eager=1 if eager else 0, precision=PRECISIONS[precision],
                 skeleton=1 if skeleton else 0)
        st = (Stats * n)()
        with torch.cuda.device(self.plans[0].device):
            _check(lib.asdsm_batch_solve(self._h, sp, gp, up, byref(o), st))
        return us, [_info(0, st[i], None, None, profile) for i in range(n)]

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load_library().asdsm_batch_destroy(self._h)
            self._h = c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Net:
    """Correction network of the learned solve (include/asdsm_learn.h) for n^3 volumes."""

    CHANNELS = 16  # stored input channels per voxel (the first 7 are read)

    def __init__(self, n, seed=0, device=None, stream=None):
        import torch
        lib = load_library()
        if not torch.cuda.is_available():
            raise RuntimeError("the correction network needs a HIP GPU; none is available")
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.n = int(n)
        self.plan = None
        self._h = c_void_p()
        with torch.cuda.device(self.device):
            _check(lib.asdsm_net_create(byref(self._h), self.n, c_uint64(int(seed) & 0xFFFFFFFFFFFFFFFF),
                                        c_void_p(self.stream.cuda_stream)))
            cnt, nbytes = c_size_t(), c_size_t()
            _check(lib.asdsm_net_param_count(self._h, byref(cnt)))
            _check(lib.asdsm_net_workspace_size(self._h, byref(nbytes)))
            self.n_params = int(cnt.value)
            self.workspace_bytes = int(nbytes.value)
            self._ws = torch.empty(self.workspace_bytes + 256, dtype=torch.uint8, device=self.device)
            aligned = (self._ws.data_ptr() + 255) // 256 * 256
            _check(lib.asdsm_net_set_workspace(self._h, c_void_p(aligned), c_size_t(self.workspace_bytes)))

    @property
    def n_vox(self) -> int:
        return self.n ** 3

    def get_params(self):
        import numpy as np
        out = np.empty(self.n_params, dtype=np.float32)
        _check(load_library().asdsm_net_params(self._h, out.ctypes.data_as(POINTER(ctypes.c_float)), 1))
        return out

    def set_params(self, params):
        import numpy as np
        a = np.ascontiguousarray(params, dtype=np.float32)
        if a.size != self.n_params:
            raise ValueError(f"expected {self.n_params} parameters, got {a.size}")
        _check(load_library().asdsm_net_params(self._h, a.ctypes.data_as(POINTER(ctypes.c_float)), 0))

    def forward(self, x, out=None):
        import torch
        if out is None:
            out = torch.empty(self.n_vox, dtype=torch.float32, device=self.device)
        with torch.cuda.device(self.device):
            _check(load_library().asdsm_net_forward(self._h, _fptr(x, self.n_vox * self.CHANNELS, "x"),
                                                    _fptr(out, self.n_vox, "out")))
        return out

    def gradient(self, x, target, loss="mse", want_grad=True, want_loss=True):
        """(loss or None, flat parameter gradient as numpy float32 or None).  Without either the
        call only enqueues the work (the gradient stays on the device for adam())."""
        import numpy as np
        import torch
        g = np.empty(self.n_params, dtype=np.float32) if want_grad else None
        lv = c_double()
        with torch.cuda.device(self.device):
            _check(load_library().asdsm_net_gradient(
                self._h, _fptr(x, self.n_vox * self.CHANNELS, "x"), _fptr(target, self.n_vox, "target"),
                NET_LOSSES[loss], byref(lv) if want_loss else None,
                g.ctypes.data_as(POINTER(ctypes.c_float)) if want_grad else None))
        return (lv.value if want_loss else None), g

    def adam(self, lr):
        import torch
        with torch.cuda.device(self.device):
            _check(load_library().asdsm_net_adam(self._h, ctypes.c_float(lr)))

    def bind(self, plan):
        import torch
        with torch.cuda.device(self.device):
            _check(load_library().asdsm_net_bind(self._h, plan._h))
        self.plan = plan

    def features(self, r, rnorm2, offset=(0, 0, 0), x=None, rhat=None):
        """Network input (n^3 x 16) and rhat (n^3) for a window of the bound plan's residual r;
        rnorm2 = ||r||_2^2 of the whole residual (Plan.residual returns ||r||_2)."""
        import torch
        if self.plan is None:
            raise RuntimeError("bind the network to a plan first")
        if x is None:
            x = torch.empty(self.n_vox * self.CHANNELS, dtype=torch.float32, device=self.device)
        if rhat is None:
            rhat = torch.empty(self.n_vox, dtype=torch.float32, device=self.device)
        off = (c_int * 3)(*[int(o) for o in offset])
        with torch.cuda.device(self.device):
            _check(load_library().asdsm_net_features(self._h, _dptr(r, self.plan.n_fine, "r"), float(rnorm2), off,
                                                     _fptr(x, self.n_vox * self.CHANNELS, "x"),
                                                     _fptr(rhat, self.n_vox, "rhat")))
        return x, rhat

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load_library().asdsm_net_destroy(self._h)
            self._h = c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def solve_learned(plan, net, s, g, u=None, factor=4.0, max_iter=50, rtol=1e-10, stag_window=3,
                  stag_eta=1e-3, resume=False, k0=0, profile=False, eager=False, precision="fp64"):
    """asdsm_solve_learned: (u, info) with info["accepted"] = accepted learned proposals."""
    import torch
    lib = load_library()
    if u is None:
        u = torch.empty(plan.n_fine, dtype=torch.float64, device=plan.device)
    o, hist, steps = _opts(max_iter, rtol, stag_window, stag_eta, resume, k0, profile, eager, precision)
    st = Stats()
    acc = c_int()
    with torch.cuda.device(plan.device):
        rc = _check(lib.asdsm_solve_learned(plan._h, net._h, float(factor), _dptr(s, plan.n_fine, "s"),
                                            _dptr(g, plan.n_faces, "g"), _dptr(u, plan.n_fine, "u"),
                                            byref(o), byref(st), byref(acc)))
    info = _info(rc, st, hist, steps, profile)
    info["accepted"] = acc.value
    return u, info


def probe_mfma_f64(iters=20000, device=0):
    """Measured FP64 MFMA rate of the device in TFLOP/s (asdsm_probe_mfma_f64)."""
    import torch
    lib = load_library()
    dev = torch.device("cuda", device)
    scratch = torch.empty(int(lib.asdsm_probe_mfma_scratch_bytes()), dtype=torch.uint8, device=dev)
    out = c_double()
    st = torch.cuda.current_stream(dev)
    with torch.cuda.device(dev):
        _check(lib.asdsm_probe_mfma_f64(c_void_p(scratch.data_ptr()), int(iters), c_void_p(st.cuda_stream),
                                        byref(out)))
    return out.value


def probe_copy(nbytes=1 << 30, reps=5, device=0):
    """Measured streaming-copy rate of the device in TB/s, reads plus writes (asdsm_probe_copy)."""
    import torch
    lib = load_library()
    dev = torch.device("cuda", device)
    src = torch.zeros(nbytes // 8, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    out = c_double()
    st = torch.cuda.current_stream(dev)
    with torch.cuda.device(dev):
        _check(lib.asdsm_probe_copy(c_void_p(src.data_ptr()), c_void_p(dst.data_ptr()), c_size_t(src.numel() * 8),
                                    int(reps), c_void_p(st.cuda_stream), byref(out)))
    return out.value
