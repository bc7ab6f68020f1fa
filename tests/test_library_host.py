"""Host-side checks of libfastdf.so that need no GPU: the library loads, exports
every symbol the header declares, validates configurations, and its FP64
schedule and sigma_8 normalisation agree with the oracle's."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2207_14256_amd import fastdf, workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(fastdf.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    return fastdf.load()


def test_exports_match_header(lib):
    header = open(os.path.join(ROOT, "include", "fastdf.h")).read()
    declared = set(re.findall(r"^(?:int|const char\*)\s+(fdf_\w+)\(", header, re.M))
    assert declared == set(fastdf.EXPORTS)
    for name in declared:
        assert hasattr(lib, name), name


def _size(cfg_struct):
    n = ctypes.c_size_t()
    return fastdf.load().fdf_workspace_size(ctypes.byref(cfg_struct), ctypes.byref(n)), n.value


@pytest.mark.parametrize("field,value", [
    ("grid_n", 48), ("grid_n", 4), ("grid_n", 2048), ("box_mpc", 0.0), ("n_steps", 0),
    ("precision", 7), ("potential_model", 9), ("abi_version", 99), ("slip_amp", 1.5),
    ("max_particles", 0), ("sort_every", -1),
])
def test_invalid_configs_rejected(lib, field, value):
    c = fastdf.make_config(workloads.preset("c1"))
    setattr(c, field, value)
    rc, _ = _size(c)
    assert rc == -1
    ctx = ctypes.c_void_p()
    assert lib.fdf_create(ctypes.byref(c), None, ctypes.byref(ctx)) == -1


def test_equal_redshifts_and_big_drift_rejected(lib):
    c = fastdf.make_config(workloads.preset("c1"))
    c.z_end = c.z_begin
    assert _size(c)[0] == -1
    # a schedule whose largest drift exceeds half a box is refused at create
    c = fastdf.make_config(workloads.preset("c1", box_mpc=50.0, n_steps=5, z_end=0.0))
    ctx = ctypes.c_void_p()
    assert lib.fdf_create(ctypes.byref(c), None, ctypes.byref(ctx)) == -1


def test_workspace_size_grows_with_capacity(lib):
    c = fastdf.make_config(workloads.preset("c1"))
    rc, s1 = _size(c)
    c.max_particles *= 2
    rc2, s2 = _size(c)
    assert rc == rc2 == 0 and s2 > s1
    c.sort_every = 20
    assert _size(c)[1] > s2


def _create(lib, cfg):
    c = fastdf.make_config(cfg)
    ctx = ctypes.c_void_p()
    assert lib.fdf_create(ctypes.byref(c), None, ctypes.byref(ctx)) == 0
    return ctx, c


@pytest.mark.parametrize("name", ["c1", "c2", "c3"])
def test_schedule_matches_oracle(lib, name):
    """The library's Gauss-Legendre step integrals equal the oracle's adaptive
    quadrature (sec. 3.3 step sizes)."""
    from oracle import pipeline
    cfg = workloads.preset(name)
    ctx, c = _create(lib, cfg)
    n = c.n_steps
    t = np.empty(5 * n + 1)
    assert lib.fdf_read_schedule(ctx, t.ctypes.data_as(ctypes.POINTER(ctypes.c_double))) == 0
    ref = pipeline.schedule(cfg)
    assert np.allclose(t[:n + 1], ref["a"], rtol=1e-14)
    assert np.allclose(t[n + 1:2 * n + 1], ref["a_half"], rtol=1e-14)
    for i, key in enumerate(("kick1", "kick2", "drift")):
        assert np.allclose(t[(2 + i) * n + 1:(3 + i) * n + 1], ref[key], rtol=1e-12), key
    lib.fdf_destroy(ctx)


def test_amplitude_and_tau_match_oracle(lib):
    from oracle import background, pipeline
    cfg = workloads.preset("c2")
    ctx, _ = _create(lib, cfg)
    info = fastdf.Info()
    assert lib.fdf_get_info(ctx, ctypes.byref(info)) == 0
    assert info.amplitude == pytest.approx(pipeline.amplitude(cfg), rel=1e-10)
    a0 = 1 / (1 + cfg["z_begin"])
    assert info.tau_begin == pytest.approx(background.conformal_time(a0, cfg["h"], 1.0), rel=1e-12)
    assert info.step_index == 0 and info.n_species == 0
    lib.fdf_destroy(ctx)


def test_calls_without_workspace_fail_cleanly(lib):
    ctx, _ = _create(lib, workloads.preset("c1"))
    fid = ctypes.c_int32()
    assert lib.fdf_add_field(ctx, 1, 0, ctypes.byref(fid)) == -3
    assert lib.fdf_step(ctx, 1) == -3
    assert b"workspace" in lib.fdf_last_error(ctx)
    assert lib.fdf_status_string(-5) == b"capacity exceeded"
    assert lib.fdf_attach_workspace(ctx, ctypes.c_void_p(12345), 10) == -3
    lib.fdf_destroy(ctx)


def test_truncate_field_is_spectral_restriction():
    """A band-limited fine field and its truncation describe the same function:
    the coarse field equals the fine one sampled on the coarse mesh."""
    from paper_2207_14256_amd.convergence import truncate_field
    rng = np.random.default_rng(4)
    G, Gc = 32, 8
    real = rng.normal(size=(G, G, G))
    dk = np.fft.rfftn(real) / G ** 3
    n = np.arange(G)
    s = np.where(n < G // 2, n, n - G)
    keep = (np.abs(s)[:, None, None] < Gc // 2) & (np.abs(s)[None, :, None] < Gc // 2) \
        & (np.arange(G // 2 + 1)[None, None, :] < Gc // 2)
    dk = np.where(keep, dk, 0)
    fine = np.fft.irfftn(dk, s=(G, G, G), axes=(0, 1, 2)) * G ** 3
    coarse = np.fft.irfftn(truncate_field(dk, Gc), s=(Gc, Gc, Gc), axes=(0, 1, 2)) * Gc ** 3
    step = G // Gc
    assert np.allclose(coarse, fine[::step, ::step, ::step], rtol=0, atol=1e-12 * np.abs(fine).max())


_CTYPES = {"int32_t": ctypes.c_int32, "int64_t": ctypes.c_int64, "double": ctypes.c_double,
           "float": ctypes.c_float, "size_t": ctypes.c_size_t}


def _header_fields(struct_name):
    """(name, ctype) of each member of `typedef struct <name> {...}` in the
    header, in order (comments stripped; `double a, b;` gives two members)."""
    header = open(os.path.join(ROOT, "include", "fastdf.h")).read()
    header = re.sub(r"/\*.*?\*/", "", header, flags=re.S)
    body = re.search(r"typedef struct %s \{(.*?)\} %s;" % (struct_name, struct_name), header, re.S).group(1)
    fields = []
    for decl in body.split(";"):
        decl = decl.strip()
        if not decl:
            continue
        ctype, names = decl.split(None, 1)
        for name in names.split(","):
            fields.append((name.strip(), _CTYPES[ctype]))
    return fields


@pytest.mark.parametrize("struct_name,cls", [("fdf_config", fastdf.Config), ("fdf_info", fastdf.Info),
                                             ("fdf_tuning", fastdf.Tuning)])
def test_binding_structs_match_header(struct_name, cls):
    """The ctypes structures of the binding have the header's members, types
    and order (a mismatch would shift every later member)."""
    assert [(n, t) for n, t in cls._fields_] == _header_fields(struct_name)
