"""The spatial re-sort permutes the particle state only: results by id are
bit-identical for any sort cadence and tile size (GPU, through the C ABI)."""
import numpy as np
import pytest

from paper_2207_14256_amd import fastdf, workloads

pytestmark = pytest.mark.gpu


def _final_state(cfg, sort_every, tiles=0, steps=None):
    cfg = dict(cfg, sort_every=sort_every)
    ctx, fields, species = fastdf.setup_workload(cfg)
    if tiles:
        ctx.set_tuning(sort_tiles=tiles)
    ctx.step(cfg["n_steps"] if steps is None else steps)
    x, q = ctx.read_state(species[0])
    w = ctx.weights(species[0]).cpu().numpy()
    ctx.close()
    return x, q, w


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_sort_cadence_invariance(prec):
    print("[gpu-case] sort cadence invariance %s" % prec, flush=True)
    cfg = workloads.small("c2", grid_n=32, n_side=29, n_steps=60, precision=prec,
                          box_mpc=600.0, z_begin=1e6, z_end=10.0)
    ref = _final_state(cfg, 0)
    for every, tiles in ((1, 0), (7, 0), (20, 4), (3, 16)):
        got = _final_state(cfg, every, tiles)
        for a, b in zip(got, ref):
            assert np.array_equal(a, b), (every, tiles)


def test_sort_then_backward_walk():
    """Sorting in both directions of a forward-backward walk keeps ids aligned."""
    print("[gpu-case] sort + backward walk", flush=True)
    cfg = workloads.small("c2", grid_n=16, n_side=20, n_steps=30, precision="fp64",
                          box_mpc=500.0, z_begin=1e6, z_end=100.0, sort_every=4)
    ctx, fields, species = fastdf.setup_workload(cfg)
    x0, q0 = ctx.read_state(species[0])
    ctx.step(30)
    ctx.step(-30)
    x1, q1 = ctx.read_state(species[0])
    L = cfg["box_mpc"]
    d = (x1 - x0 + L / 2) % L - L / 2
    assert np.max(np.abs(d)) < 1e-10 * L
    assert np.max(np.abs(q1 - q0)) < 1e-10 * np.max(np.abs(q0))
    ctx.close()


def _state_by_id(cfg, tuning, steps=None, back=0):
    ctx, fields, species = fastdf.setup_workload(cfg, tuning=tuning)
    ctx.step(cfg["n_steps"] if steps is None else steps)
    if back:
        ctx.step(-back)
    out = []
    for s in species:
        x, q = ctx.read_state(s)
        out += [x, q, ctx.weights(s).cpu().numpy()]
    ctx.close()
    return out


FUSED_CASES = {
    # two species with ragged counts (not multiples of the 1024-particle rank block)
    "slip-8slot-two-species": dict(
        base=dict(grid_n=32, n_side=29, n_steps=60, box_mpc=600.0, z_begin=1e6, z_end=10.0),
        second=23, tuning=dict(sort_every=3)),
    # super-steps (two blended grid sets), TSC, 4-slot grids, adaptive cadence
    "radmat-superstep-tsc": dict(
        base=dict(grid_n=16, n_side=13, n_steps=60, box_mpc=600.0, z_begin=1e6, z_end=10.0,
                  model="radmat", omega_m=0.9999, omega_r=1e-4, slip_amp=0.0,
                  superstep_tol=0.01, interp_order=2),
        second=0, tuning=dict(sort_every=1, sort_cells=0.3)),
    # super-steps with CIC: the grouped two-set gathers of both push kernels
    "radmat-superstep-cic": dict(
        base=dict(grid_n=16, n_side=21, n_steps=60, box_mpc=600.0, z_begin=1e6, z_end=10.0,
                  model="radmat", omega_m=0.9999, omega_r=1e-4, slip_amp=0.01,
                  superstep_tol=0.01, interp_order=1),
        second=0, tuning=dict(sort_every=1, sort_cells=0.3, particles_per_thread=8)),
    # graph capture and replay of the fused launches
    "graph": dict(
        base=dict(grid_n=32, n_side=21, n_steps=60, box_mpc=600.0, z_begin=1e6, z_end=10.0),
        second=0, tuning=dict(sort_every=2, use_graph=1)),
}


@pytest.mark.parametrize("case", sorted(FUSED_CASES))
def test_fused_sort_push_bit_identical(case):
    """A re-sort carried out by the push (sort_fused) gives the same state by id,
    bit for bit, as separate rank/move passes and as no sorting at all."""
    print("[gpu-case] fused sort+push %s" % case, flush=True)
    spec = FUSED_CASES[case]
    cfg = workloads.small("c2", precision="fp32", **spec["base"])
    cfg["sort_every"] = 1
    if spec["second"]:
        cfg["fields"] = cfg["fields"] + [cfg["fields"][0] + 1]
        cfg["species"].append(dict(field=1, m=0.2, n_side=spec["second"], seed=2999))
    plain = _state_by_id(cfg, dict(sort_every=0))
    sep = _state_by_id(cfg, dict(spec["tuning"], sort_fused=0))
    fused = _state_by_id(cfg, dict(spec["tuning"], sort_fused=1))
    for i, (a, b, c) in enumerate(zip(plain, sep, fused)):
        assert np.array_equal(a, b), (case, i)
        assert np.array_equal(a, c), (case, i)


def test_fused_sort_backward_walk():
    """Fused re-sorts in both directions of a forward-backward walk: ids stay
    aligned and the state matches the unsorted walk bit for bit."""
    print("[gpu-case] fused sort+push backward walk", flush=True)
    cfg = workloads.small("c2", grid_n=32, n_side=24, n_steps=60, precision="fp32",
                          box_mpc=600.0, z_begin=1e6, z_end=10.0)
    cfg["sort_every"] = 1
    plain = _state_by_id(cfg, dict(sort_every=0), steps=60, back=35)
    fused = _state_by_id(cfg, dict(sort_every=3, sort_fused=1), steps=60, back=35)
    for i, (a, b) in enumerate(zip(plain, fused)):
        assert np.array_equal(a, b), i


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_launch_shape_invariance(prec):
    """Particles per thread and the cap on resident waves change only the
    launch: the state by id is bit-identical."""
    print("[gpu-case] launch shape invariance %s" % prec, flush=True)
    cfg = workloads.small("c2", grid_n=32, n_side=27, n_steps=60, precision=prec,
                          box_mpc=600.0, z_begin=1e6, z_end=10.0)
    cfg["sort_every"] = 1
    ref = _state_by_id(cfg, dict(sort_every=4))
    for ppt, waves in ((2, 3), (4, 2), (1, 8), (8, 4)):
        got = _state_by_id(cfg, dict(sort_every=4, particles_per_thread=ppt, push_waves=waves))
        for i, (a, b) in enumerate(zip(ref, got)):
            assert np.array_equal(a, b), (ppt, waves, i)


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_first_sort_of_modified_states(prec):
    """The job's first sort re-samples untouched species by id; species whose
    state was changed before it (pre-initial conditions) move their state.
    Both give the unsorted run's state by id, bit for bit."""
    print("[gpu-case] first sort, pre-IC species %s" % prec, flush=True)
    cfg = workloads.small("c2", grid_n=32, n_side=21, n_steps=60, precision=prec,
                          box_mpc=600.0, z_begin=1e6, z_end=10.0, pre_ic=True)
    cfg["sort_every"] = 1
    ref = _state_by_id(cfg, dict(sort_every=0))
    got = _state_by_id(cfg, dict(sort_every=3))
    for i, (a, b) in enumerate(zip(ref, got)):
        assert np.array_equal(a, b), i


@pytest.mark.parametrize("eom", ["exact", "canonical"])
def test_launch_shape_invariance_other_eoms(eom):
    """The cap on resident waves and the particles per thread apply to the
    kernels of the other equations of motion as well; their results by id do
    not change either."""
    print("[gpu-case] launch shape invariance eom=%s" % eom, flush=True)
    cfg = workloads.small("c2", grid_n=16, n_side=15, n_steps=60, precision="fp32",
                          box_mpc=600.0, z_begin=1e6, z_end=10.0, eom=eom)
    cfg["sort_every"] = 1
    ref = _state_by_id(cfg, dict(sort_every=4))
    for ppt, waves in ((2, 3), (4, 2), (1, 8)):
        got = _state_by_id(cfg, dict(sort_every=4, particles_per_thread=ppt, push_waves=waves))
        for i, (a, b) in enumerate(zip(ref, got)):
            assert np.array_equal(a, b), (eom, ppt, waves, i)


@pytest.mark.parametrize("prec,fused", [("fp32", 1), ("fp32", 0), ("fp64", 0)])
def test_per_species_cadence_bit_identical(prec, fused):
    """Species of different masses re-sort on their own adaptive cadence (the
    light species far more often), in split calls, graph replay and a
    backward walk: every species' state by id equals the never-sorted run's."""
    print("[gpu-case] per-species cadence %s fused=%d" % (prec, fused), flush=True)
    cfg = workloads.small("c4", grid_n=32, n_side=0, n_steps=80, precision=prec, box_mpc=768.0,
                          z_begin=1e9, z_end=31.0, sort_every=1, sort_cells=0.0)
    cfg["fields"] = [1004, 1104]
    cfg["species"] = [dict(field=0, m=0.005, n_side=11, seed=2040),
                      dict(field=0, m=0.0502, n_side=17, seed=2042),
                      dict(field=1, m=0.05, n_side=9, seed=2044)]
    ref = _state_by_id(dict(cfg, sort_every=0), dict(sort_every=0))
    base = dict(sort_every=1, sort_cells=0.7, sort_fused=fused)
    for tuning, steps, back in ((base, None, 0), (dict(base, use_graph=1), None, 0),
                                (dict(base, particles_per_thread=1), None, 0)):
        got = _state_by_id(cfg, tuning, steps, back)
        for a, b in zip(got, ref):
            assert np.array_equal(a, b), tuning
    # split calls and a walk back to the middle
    ctx, fields, species = fastdf.setup_workload(cfg, tuning=base)
    for k in (13, 29, 38):
        ctx.step(k)
    ctx.step(-40)
    mid = []
    for s in species:
        x, q = ctx.read_state(s)
        mid += [x, q]
    ctx.close()
    ref_mid = _state_by_id(dict(cfg, sort_every=0), dict(sort_every=0), steps=40)
    ref_mid = [v for i, v in enumerate(ref_mid) if i % 3 != 2]
    L = cfg["box_mpc"]
    for i, (a, b) in enumerate(zip(mid, ref_mid)):
        if i % 2 == 0:
            assert np.max(np.abs((a - b + L / 2) % L - L / 2)) < 1e-6 * L   # ids stay aligned
        else:
            assert np.max(np.abs(a - b)) <= 1e-5 * np.max(np.abs(b))


@pytest.mark.parametrize("order", [1, 2])
def test_padded_mesh_bit_identical(order):
    """12-byte bfloat16 cells (the default) hold the same six gradient values
    as the 16-byte cells with a zero slot and a pad (pad_mesh): every particle's state,
    its weight and the spectra come out bit for bit the same, with plain and
    fused re-sorts and with CIC or TSC gathers."""
    print("[gpu-case] padded mesh order %d" % order, flush=True)
    cfg = workloads.small("c3", grid_n=32, n_side=30, n_steps=200, z_begin=1e9, z_end=3.0,
                          sort_every=4, sort_cells=0.0, interp_order=order)
    out = []
    for pad in (False, True):
        ctx, fields, species = fastdf.setup_workload(dict(cfg, pad_mesh=pad))
        ctx.step(cfg["n_steps"])
        x, q = ctx.read_state(species[0])
        w = ctx.weights(species[0]).cpu().numpy()
        g = ctx.read_grid(fields[0], 4)
        k, p, nm = ctx.power_spectrum(species, 16)
        ctx.close()
        out.append((x, q, w, g, p))
    for a, b in zip(*out):
        assert np.array_equal(a, b, equal_nan=True)


@pytest.mark.parametrize("ppt", [4, 8])
def test_sort_keys_from_push_bit_identical(ppt):
    """With one species, the push before each re-sort writes the sort keys
    (sort_keys_push): every result by id equals the run whose rank passes
    compute the keys and the never-sorted run, for a particle count that is
    not a multiple of the rank block, in one call and in split calls (the
    first re-sort of a call computes its keys itself)."""
    print("[gpu-case] sort keys from push ppt=%d" % ppt, flush=True)
    cfg = workloads.small("c3", grid_n=32, n_side=37, n_steps=200, z_begin=1e9, z_end=3.0)
    ref = _state_by_id(dict(cfg, sort_every=0), dict(sort_every=0))
    base = dict(sort_every=1, sort_cells=0.7, particles_per_thread=ppt)
    for keys in (1, 0):
        got = _state_by_id(cfg, dict(base, sort_keys_push=keys))
        for a, b in zip(got, ref):
            assert np.array_equal(a, b), keys
    # split calls (each call applies its closing half-kick on its own, so the
    # reference is the never-sorted run split the same way)
    split = {}
    for key, c, t in (("ref", dict(cfg, sort_every=0), dict(sort_every=0)),
                      ("keys", cfg, dict(base, sort_keys_push=1))):
        ctx, fields, species = fastdf.setup_workload(c, tuning=t)
        for k in (37, 63, 100):
            ctx.step(k)
        x, q = ctx.read_state(species[0])
        split[key] = (x, q, ctx.weights(species[0]).cpu().numpy())
        ctx.close()
    for a, b in zip(split["keys"], split["ref"]):
        assert np.array_equal(a, b)
