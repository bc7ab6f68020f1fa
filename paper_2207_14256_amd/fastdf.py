"""ctypes binding of libfastdf.so (argument marshalling only).

Every step of the method runs in the library's HIP kernels; this module only
converts Python values to the C ABI of ``include/fastdf.h`` and back.  PyTorch
supplies the device workspace and the stream.  Loading fails loudly when the
library has not been built: there is no fallback implementation.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfastdf.so")

ABI_VERSION = 1
PREC_FP64, PREC_FP32 = 0, 1
MODEL_POISSON, MODEL_RADMAT = 0, 1
EOMS = dict(separable=0, exact=1, canonical=2, sr_newton=3, simple_q=4, newtonian=5)   # fdf_config.eom
PK_CROSS, PK_AUTO = 0, 1
PK_DENSITY, PK_MOMENTUM = 0, 1
SPECIES_PRE_IC = 1
KERNEL_PUSH, KERNEL_SORT, KERNEL_GRID, KERNEL_INIT, KERNEL_OUTPUT = range(5)
KERNEL_CLASSES = {"push": 0, "sort": 1, "grid": 2, "init": 3, "output": 4, "push_sort": 5}

# every symbol the header declares
EXPORTS = [
    "fdf_workspace_size", "fdf_create", "fdf_attach_workspace", "fdf_reset", "fdf_destroy",
    "fdf_add_field", "fdf_set_field", "fdf_init_species", "fdf_set_species_state",
    "fdf_build_potential_grids", "fdf_step", "fdf_weights", "fdf_density_power_spectrum",
    "fdf_momentum_power_spectrum", "fdf_force_terms", "fdf_power_spectrum",
    "fdf_read_state", "fdf_read_grid", "fdf_read_field", "fdf_read_density",
    "fdf_read_schedule", "fdf_get_info", "fdf_sync", "fdf_timing_enable",
    "fdf_read_timing", "fdf_timing_reset", "fdf_status_string", "fdf_last_error",
    "fdf_get_tuning", "fdf_set_tuning", "fdf_power_spectrum_noalloc", "fdf_read_work",
]


class Config(ctypes.Structure):
    _fields_ = [
        ("abi_version", ctypes.c_int32), ("grid_n", ctypes.c_int32),
        ("box_mpc", ctypes.c_double), ("h", ctypes.c_double),
        ("omega_m", ctypes.c_double), ("omega_r", ctypes.c_double), ("omega_l", ctypes.c_double),
        ("z_begin", ctypes.c_double), ("z_end", ctypes.c_double),
        ("n_steps", ctypes.c_int32), ("precision", ctypes.c_int32),
        ("potential_model", ctypes.c_int32), ("eom", ctypes.c_int32),
        ("slip_amp", ctypes.c_double), ("slip_k", ctypes.c_double),
        ("ns", ctypes.c_double), ("sigma8", ctypes.c_double), ("gamma", ctypes.c_double),
        ("sort_every", ctypes.c_int32), ("max_fields", ctypes.c_int32),
        ("max_species", ctypes.c_int32), ("interp_order", ctypes.c_int32),
        ("max_particles", ctypes.c_int64), ("superstep_tol", ctypes.c_double),
        ("pad_mesh", ctypes.c_int32),
    ]


class Info(ctypes.Structure):
    _fields_ = [
        ("step_index", ctypes.c_int32), ("n_steps", ctypes.c_int32),
        ("a_current", ctypes.c_double), ("amplitude", ctypes.c_double),
        ("tau_begin", ctypes.c_double), ("n_fields", ctypes.c_int32),
        ("n_species", ctypes.c_int32), ("n_particles", ctypes.c_int64),
        ("workspace_used", ctypes.c_size_t),
    ]


class Tuning(ctypes.Structure):
    _fields_ = [("particles_per_thread", ctypes.c_int32), ("sort_tiles", ctypes.c_int32),
                ("sort_every", ctypes.c_int32), ("sort_cells", ctypes.c_float),
                ("persistent_blocks", ctypes.c_int32), ("use_graph", ctypes.c_int32),
                ("sort_predict", ctypes.c_int32),
                ("sort_fused", ctypes.c_int32),
                ("push_waves", ctypes.c_int32), ("sort_push_ppt", ctypes.c_int32),
                ("sort_keys_push", ctypes.c_int32)]


class FastDFError(RuntimeError):
    pass


_lib = None


def load():
    """Load libfastdf.so (built in-tree by ``paper_2207_14256_amd/build.py``)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise FastDFError("libfastdf.so not built: run __graft_entry__.build() "
                          "(hipcc, gfx950) before using the HIP path")
    lib = ctypes.CDLL(LIB_PATH)
    P, I32, I64, U64, D = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64,
                           ctypes.c_uint64, ctypes.c_double)
    PD = ctypes.POINTER(ctypes.c_double)
    sig = {
        "fdf_workspace_size": [ctypes.POINTER(Config), ctypes.POINTER(ctypes.c_size_t)],
        "fdf_create": [ctypes.POINTER(Config), P, ctypes.POINTER(P)],
        "fdf_attach_workspace": [P, P, ctypes.c_size_t],
        "fdf_reset": [P], "fdf_destroy": [P],
        "fdf_add_field": [P, U64, I32, ctypes.POINTER(I32)],
        "fdf_set_field": [P, PD, ctypes.POINTER(I32)],
        "fdf_init_species": [P, I32, D, I64, U64, I32, ctypes.POINTER(I32)],
        "fdf_set_species_state": [P, I32, D, I64, ctypes.POINTER(ctypes.c_uint32),
                                  ctypes.POINTER(ctypes.c_float), ctypes.POINTER(I32)],
        "fdf_build_potential_grids": [P, I32, D],
        "fdf_step": [P, I32],
        "fdf_weights": [P, I32, P],
        "fdf_density_power_spectrum": [P, ctypes.POINTER(I32), I32, I32, I32, PD, PD, PD],
        "fdf_momentum_power_spectrum": [P, ctypes.POINTER(I32), I32, I32, I32, PD, PD, PD],
        "fdf_force_terms": [P, I32, PD],
        "fdf_power_spectrum": [P, ctypes.POINTER(I32), I32, I32, I32, I32, I32, PD, PD, PD],
        "fdf_power_spectrum_noalloc": [P, ctypes.POINTER(I32), I32, I32, I32, I32, I32, P],
        "fdf_read_state": [P, I32, PD, PD],
        "fdf_read_grid": [P, I32, I32, PD],
        "fdf_read_field": [P, I32, PD],
        "fdf_read_density": [P, I32, PD],
        "fdf_read_schedule": [P, PD],
        "fdf_get_info": [P, ctypes.POINTER(Info)],
        "fdf_sync": [P], "fdf_timing_enable": [P, I32],
        "fdf_read_timing": [P, I32, PD, ctypes.POINTER(I64)],
        "fdf_timing_reset": [P],
        "fdf_read_work": [P, I32, ctypes.POINTER(I64)],
        "fdf_get_tuning": [P, ctypes.POINTER(Tuning)],
        "fdf_set_tuning": [P, ctypes.POINTER(Tuning)],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    lib.fdf_status_string.argtypes = [ctypes.c_int]
    lib.fdf_status_string.restype = ctypes.c_char_p
    lib.fdf_last_error.argtypes = [P]
    lib.fdf_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def make_config(cfg):
    """fdf_config from a workload dict (see workloads.py) plus capacities."""
    n_particles = sum(int(sp.get("n", sp["n_side"] ** 3)) for sp in cfg["species"])
    c = Config()
    c.abi_version = ABI_VERSION
    c.grid_n = int(cfg["grid_n"])
    c.box_mpc = float(cfg["box_mpc"])
    c.h = float(cfg["h"])
    c.omega_m = float(cfg["omega_m"])
    c.omega_r = float(cfg.get("omega_r", 0.0))
    c.omega_l = float(cfg.get("omega_l", 0.0))
    c.z_begin = float(cfg["z_begin"])
    c.z_end = float(cfg["z_end"])
    c.n_steps = int(cfg["n_steps"])
    c.precision = PREC_FP64 if cfg["precision"] == "fp64" else PREC_FP32
    c.potential_model = {"poisson": MODEL_POISSON, "radmat": MODEL_RADMAT}[cfg["model"]]
    c.slip_amp = float(cfg.get("slip_amp", 0.0))
    c.slip_k = float(cfg.get("slip_k", 1.0))
    c.ns = float(cfg["ns"])
    c.sigma8 = float(cfg["sigma8"])
    c.gamma = float(cfg["gamma"])
    c.sort_every = int(cfg.get("sort_every", 0))
    c.max_fields = int(cfg.get("max_fields", len(cfg["fields"])))
    c.max_species = int(cfg.get("max_species", len(cfg["species"])))
    c.max_particles = int(cfg.get("max_particles", n_particles))
    c.superstep_tol = float(cfg.get("superstep_tol", 0.0))
    c.pad_mesh = int(bool(cfg.get("pad_mesh", False)))
    c.eom = EOMS[cfg.get("eom", "separable")]
    c.interp_order = int(cfg.get("interp_order", 1))
    return c


def workspace_size(cfg):
    lib = load()
    n = ctypes.c_size_t()
    rc = lib.fdf_workspace_size(ctypes.byref(make_config(cfg)), ctypes.byref(n))
    if rc:
        raise FastDFError("invalid configuration (status %d)" % rc)
    return n.value


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


class Context:
    """One fdf_ctx with a torch-allocated workspace on the current HIP device."""

    def __init__(self, cfg, device="cuda", stream=None):
        import torch
        self.lib = load()
        self.cfg = cfg
        self.ccfg = make_config(cfg)
        self.torch = torch
        self.device = torch.device(device)
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        ctx = ctypes.c_void_p()
        self._check(self.lib.fdf_create(ctypes.byref(self.ccfg), ctypes.c_void_p(stream.cuda_stream),
                                        ctypes.byref(ctx)), "fdf_create", ctx=None)
        self.ctx = ctx
        self._species_n = {}
        size = workspace_size(cfg)
        # 256-byte aligned: torch's caching allocator returns at least 512-byte alignment
        self.workspace = torch.empty(size, dtype=torch.uint8, device=self.device)
        self._check(self.lib.fdf_attach_workspace(self.ctx, ctypes.c_void_p(self.workspace.data_ptr()),
                                                  size), "fdf_attach_workspace")

    # ---------------------------------------------------------------- errors --
    def _check(self, rc, what, ctx=0):
        if rc != 0:
            c = self.ctx if ctx == 0 else ctx
            msg = self.lib.fdf_last_error(c).decode() if c else ""
            raise FastDFError("%s failed: %s (%d) %s" % (
                what, self.lib.fdf_status_string(rc).decode(), rc, msg))

    def close(self):
        if getattr(self, "ctx", None):
            self.lib.fdf_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---------------------------------------------------------------- inputs --
    def reset(self):
        self._check(self.lib.fdf_reset(self.ctx), "fdf_reset")
        self._species_n = {}

    def add_field(self, seed, fixed_amp=False):
        fid = ctypes.c_int32()
        self._check(self.lib.fdf_add_field(self.ctx, int(seed), int(bool(fixed_amp)), ctypes.byref(fid)),
                    "fdf_add_field")
        return fid.value

    def set_field(self, delta_k):
        G = self.ccfg.grid_n
        a = np.ascontiguousarray(delta_k, dtype=np.complex128)
        assert a.shape == (G, G, G // 2 + 1)
        buf = np.ascontiguousarray(a.view(np.float64))
        fid = ctypes.c_int32()
        self._check(self.lib.fdf_set_field(self.ctx, _dptr(buf), ctypes.byref(fid)), "fdf_set_field")
        return fid.value

    def init_species(self, field, m, n, seed, pre_ic=False):
        sid = ctypes.c_int32()
        self._check(self.lib.fdf_init_species(self.ctx, int(field), float(m), int(n), int(seed),
                                              SPECIES_PRE_IC if pre_ic else 0, ctypes.byref(sid)),
                    "fdf_init_species")
        self._species_n[sid.value] = int(n)
        return sid.value

    def set_species_state(self, field, m, xu, q):
        xu = np.ascontiguousarray(xu, dtype=np.uint32)
        q = np.ascontiguousarray(q, dtype=np.float32)
        n = xu.shape[0]
        assert xu.shape == (n, 3) and q.shape == (n, 3)
        sid = ctypes.c_int32()
        self._check(self.lib.fdf_set_species_state(
            self.ctx, int(field), float(m), n, xu.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)),
            q.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), ctypes.byref(sid)), "fdf_set_species_state")
        self._species_n[sid.value] = int(n)
        return sid.value

    # -------------------------------------------------------------- hot path --
    def build_potential_grids(self, field, a):
        self._check(self.lib.fdf_build_potential_grids(self.ctx, int(field), float(a)),
                    "fdf_build_potential_grids")

    def step(self, n):
        self._check(self.lib.fdf_step(self.ctx, int(n)), "fdf_step")

    def weights(self, species, out=None):
        n = self.n_particles(species)
        if out is None:
            out = self.torch.empty(n, dtype=self.torch.float64, device=self.device)
        assert out.dtype == self.torch.float64 and out.numel() >= n and out.is_contiguous()
        self._check(self.lib.fdf_weights(self.ctx, int(species), ctypes.c_void_p(out.data_ptr())),
                    "fdf_weights")
        return out

    def power_spectrum(self, species, n_bins, mode="cross", quantity="density", analysis_n=0):
        """(mean k, P(k), modes) of the energy density ('density') or of the
        momentum perturbation (1 + delta) theta ('momentum'), on the mesh G or
        an analysis mesh of analysis_n points per side."""
        sp = np.asarray(species if hasattr(species, "__len__") else [species], dtype=np.int32)
        k = np.empty(n_bins)
        p = np.empty(n_bins)
        nm = np.empty(n_bins)
        spp = sp.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        md = PK_AUTO if mode == "auto" else PK_CROSS
        if analysis_n:
            qn = {"density": PK_DENSITY, "momentum": PK_MOMENTUM}[quantity]
            self._check(self.lib.fdf_power_spectrum(self.ctx, spp, len(sp), int(n_bins), md, qn,
                                                    int(analysis_n), _dptr(k), _dptr(p), _dptr(nm)),
                        "fdf_power_spectrum")
        else:
            name = {"density": "fdf_density_power_spectrum", "momentum": "fdf_momentum_power_spectrum"}[quantity]
            self._check(getattr(self.lib, name)(self.ctx, spp, len(sp), int(n_bins), md,
                                                _dptr(k), _dptr(p), _dptr(nm)), name)
        return k, p, nm

    def power_spectrum_noalloc(self, species, n_bins, out, mode="cross", quantity="density",
                               analysis_n=0):
        """fdf_power_spectrum_noalloc: the spectrum on an analysis mesh of at
        most 64^3, written to the device tensor out (3 * n_bins float64:
        mean k, P(k), modes) without any allocation; asynchronous."""
        sp = np.asarray(species if hasattr(species, "__len__") else [species], dtype=np.int32)
        assert out.dtype == self.torch.float64 and out.is_contiguous() and out.numel() >= 3 * n_bins
        md = PK_AUTO if mode == "auto" else PK_CROSS
        qn = {"density": PK_DENSITY, "momentum": PK_MOMENTUM}[quantity]
        self._check(self.lib.fdf_power_spectrum_noalloc(
            self.ctx, sp.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), len(sp), int(n_bins), md, qn,
            int(analysis_n), ctypes.c_void_p(out.data_ptr())), "fdf_power_spectrum_noalloc")
        return out

    def force_terms(self, species):
        """rms magnitudes of the four terms of eq. releq at the current state:
        (Newtonian, q^2 grad phi, q (q.grad phi), q phidot) in eV/Mpc."""
        out = np.empty(4)
        self._check(self.lib.fdf_force_terms(self.ctx, int(species), _dptr(out)), "fdf_force_terms")
        return out

    # ------------------------------------------------------------- read-back --
    def info(self):
        inf = Info()
        self._check(self.lib.fdf_get_info(self.ctx, ctypes.byref(inf)), "fdf_get_info")
        return inf

    def n_particles(self, species):
        return self._species_n[species]

    def read_state(self, species):
        n = self._species_n[species]
        x = np.empty((n, 3))
        q = np.empty((n, 3))
        self._check(self.lib.fdf_read_state(self.ctx, int(species), _dptr(x), _dptr(q)), "fdf_read_state")
        return x, q

    def read_grid(self, field, slot):
        G = self.ccfg.grid_n
        g = np.empty((G, G, G))
        self._check(self.lib.fdf_read_grid(self.ctx, int(field), int(slot), _dptr(g)), "fdf_read_grid")
        return g

    def read_field(self, field):
        G = self.ccfg.grid_n
        d = np.empty((G, G, G // 2 + 1), dtype=np.complex128)
        buf = d.view(np.float64)
        self._check(self.lib.fdf_read_field(self.ctx, int(field), _dptr(buf)), "fdf_read_field")
        return d

    def read_density(self, half):
        G = self.ccfg.grid_n
        g = np.empty((G, G, G))
        self._check(self.lib.fdf_read_density(self.ctx, int(half), _dptr(g)), "fdf_read_density")
        return g

    def read_schedule(self):
        n = self.ccfg.n_steps
        t = np.empty(5 * n + 1)
        self._check(self.lib.fdf_read_schedule(self.ctx, _dptr(t)), "fdf_read_schedule")
        return dict(a=t[:n + 1], a_half=t[n + 1:2 * n + 1], kick1=t[2 * n + 1:3 * n + 1],
                    kick2=t[3 * n + 1:4 * n + 1], drift=t[4 * n + 1:])

    def get_tuning(self):
        t = Tuning()
        self._check(self.lib.fdf_get_tuning(self.ctx, ctypes.byref(t)), "fdf_get_tuning")
        return dict(particles_per_thread=t.particles_per_thread, sort_tiles=t.sort_tiles,
                    sort_every=t.sort_every, sort_cells=t.sort_cells,
                    persistent_blocks=t.persistent_blocks, use_graph=t.use_graph,
                    sort_predict=t.sort_predict, sort_fused=t.sort_fused, push_waves=t.push_waves,
                    sort_push_ppt=t.sort_push_ppt, sort_keys_push=t.sort_keys_push)

    def set_tuning(self, **kw):
        cur = self.get_tuning()
        cur.update(kw)
        t = Tuning(cur["particles_per_thread"], cur["sort_tiles"], cur["sort_every"],
                   float(cur["sort_cells"]), int(cur["persistent_blocks"]), int(cur["use_graph"]),
                   int(cur["sort_predict"]), int(cur["sort_fused"]), int(cur["push_waves"]),
                   int(cur.get("sort_push_ppt", 4)), int(cur.get("sort_keys_push", 1)))
        self._check(self.lib.fdf_set_tuning(self.ctx, ctypes.byref(t)), "fdf_set_tuning")

    def sync(self):
        self._check(self.lib.fdf_sync(self.ctx), "fdf_sync")

    def timing(self, enable=True):
        self._check(self.lib.fdf_timing_enable(self.ctx, int(bool(enable))), "fdf_timing_enable")

    def read_timing(self, kernel):
        ms = ctypes.c_double()
        n = ctypes.c_int64()
        cls = KERNEL_CLASSES[kernel] if isinstance(kernel, str) else int(kernel)
        self._check(self.lib.fdf_read_timing(self.ctx, cls, ctypes.byref(ms), ctypes.byref(n)),
                    "fdf_read_timing")
        return ms.value, n.value

    def read_work(self, kernel_class):
        """(particle-updates with a drift, kick-only updates, mesh cells read)
        of the timed launches of a kernel class."""
        w = (ctypes.c_int64 * 3)()
        self._check(self.lib.fdf_read_work(self.ctx, KERNEL_CLASSES[kernel_class], w), "fdf_read_work")
        return int(w[0]), int(w[1]), int(w[2])

    def timing_reset(self):
        self._check(self.lib.fdf_timing_reset(self.ctx), "fdf_timing_reset")


def setup_workload(cfg, device="cuda", ctx=None, tuning=None):
    """Create (or reset) a context and add the workload's fields and species;
    tuning (a dict for Context.set_tuning) is applied when given.

    Returns (ctx, field_ids, species_ids)."""
    if ctx is None:
        ctx = Context(cfg, device)
    else:
        ctx.reset()
    if tuning:
        ctx.set_tuning(**tuning)
    elif cfg.get("sort_cells", 0.0) > 0 and cfg.get("sort_every", 0) > 0:
        ctx.set_tuning(sort_cells=float(cfg["sort_cells"]))
    fields = [ctx.add_field(seed, cfg.get("fixed_amp", False)) for seed in cfg["fields"]]
    species = []
    for sp in cfg["species"]:
        n = int(sp.get("n", sp["n_side"] ** 3))
        species.append(ctx.init_species(fields[sp["field"]], sp["m"], n, sp["seed"],
                                        cfg.get("pre_ic", False)))
    return ctx, fields, species
