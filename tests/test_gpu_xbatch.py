"""GPU tests of batched periodic boxes (graph of per-step kernel nodes,
persistent kernel with grid barrier launched directly or from a graph,
per-step launches).  Collected after the other GPU tests.

* every mode gives the same bits, under every schedule (tile size, resident
  blocks per CU, tiles per draw);
* an item evolves bit for bit as a single context of the same configuration;
* an item matches the FP64 oracle to the FP32 bar;
* the full workload (256 homogenized unit cells, edges 32..96, 2000 steps)
  runs in one graph launch and gives positive, finite permeabilities.
"""
import os

import numpy as np
import pytest

import oracle
from oracle import OracleConfig
from paper_2310_14746_amd import inputs
from tests._parity import rel_l2_drho, rel_l2_u

pytestmark = pytest.mark.gpu
NT = max(1, min(16, os.cpu_count() or 1))


def say(msg):
    print(f"[gpu-batch] {msg}", flush=True)


@pytest.fixture(scope="module")
def H():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2310_14746_amd import hlbm
    hlbm.load()
    return hlbm


ITEMS = [
    dict(shape=(32, 32, 32), tau=0.6, force=(1e-5, 0, 0)),
    dict(shape=(48, 40, 24), tau=0.9, force=(0, 2e-5, 0)),
    dict(shape=(20, 36, 28), tau=0.55, force=(1e-5, 1e-5, 0)),   # ragged last tile
    dict(shape=(64, 8, 12), tau=0.75, force=(0, 0, 3e-5)),
]


def _fields(items, seed=0):
    out = []
    for k, it in enumerate(items):
        nx, ny, nz = it["shape"]
        d = inputs.periodic_smooth(inputs.uniform_noise((nz, ny, nx), seed + k), 1.0, 3)
        out.append(inputs.round_to(d, "f32").astype(np.float32).ravel())
    return out


def _run_batch(H, items, fields, steps, mode, **sched):
    b = H.HLBMBatch(items, "f32", mode=mode, **sched)
    try:
        for k, d in enumerate(fields):
            b.set_porosity(k, d)
        b.step(steps)
        b.sync()
        st, s = b.get_state()
        mom = [tuple(t.cpu().numpy() for t in b.moments(k)) for k in range(len(items))]
        return st.cpu().numpy(), mom, b.totals()
    finally:
        b.close()


def _run_single(H, it, d, steps):
    sim = H.HLBM(19, "f32", it["shape"], tau=it["tau"], force=it["force"])
    try:
        sim.set_porosity(d)
        sim.step(steps)
        drho, u, tot = sim.moments("f64", totals=True)
        st, _ = sim.get_state()
        return st.cpu().numpy(), (drho.cpu().numpy(), u.cpu().numpy()), tot
    finally:
        sim.close()


def test_single_item_batch_equals_single_context(H):
    it = dict(shape=(40, 24, 16), tau=0.7, force=(1e-5, 0, 0))
    d = _fields([it], 7)[0]
    ref_state, _, _ = _run_single(H, it, d, 30)
    for mode in ("per_step", "persistent", "graph", "graph_persistent"):
        say(f"one item, mode {mode}")
        st, _, _ = _run_batch(H, [it], [d], 30, mode)
        assert np.array_equal(st, ref_state), mode


def test_modes_bitwise_and_items_match_single_contexts(H):
    fields = _fields(ITEMS, 3)
    steps = 41
    ref = None
    for mode in ("per_step", "persistent", "graph", "graph_persistent"):
        say(f"{len(ITEMS)} items, mode {mode}, {steps} steps")
        st, mom, tot = _run_batch(H, ITEMS, fields, steps, mode)
        if ref is None:
            ref = (st, mom, tot)
        else:
            assert np.array_equal(st, ref[0]), mode
            assert np.array_equal(tot, ref[2]), mode
    for k, it in enumerate(ITEMS):
        _, (dr, u), tot_s = _run_single(H, it, fields[k], steps)
        assert np.array_equal(ref[1][k][0], dr) and np.array_equal(ref[1][k][1], u), k
        assert np.allclose(ref[2][k], tot_s, rtol=1e-12, atol=1e-18), k


@pytest.mark.parametrize("tile,bpc,chunk", [(64, 0, 1), (128, 1, 3), (256, 0, 0), (256, -1, 2),
                                            (320, 1, 1), (512, 1, 1), (512, 0, 7)])
def test_schedules_bitwise(H, tile, bpc, chunk):
    """Every tile size, resident-block count and chunk gives the state of the
    default per-step run bit for bit (ragged last tiles included); bpc -1 = all
    that fit."""
    fields = _fields(ITEMS, 11)
    steps = 23
    ref, _, ref_tot = _run_batch(H, ITEMS, fields, steps, "per_step")
    for mode in ("graph", "graph_persistent", "persistent", "per_step"):
        b = H.HLBMBatch(ITEMS, "f32", mode=mode, tile=tile)
        try:
            sc = b.schedule()
            b.set_schedule(sc["max_blocks_per_cu"] if bpc < 0 else bpc, chunk)
            sc = b.schedule()
            say(f"schedule {sc}, mode {mode}")
            assert sc["tile"] == tile and 1 <= sc["blocks_per_cu"] <= sc["max_blocks_per_cu"]
            assert sc["chunk"] == (chunk or 2)
            for k, d in enumerate(fields):
                b.set_porosity(k, d)
            b.step(steps)
            b.sync()
            st = b.get_state()[0].cpu().numpy()
            tot = b.totals()
        finally:
            b.close()
        assert np.array_equal(st, ref), (mode, sc)
        # totals sum per-tile partials: the same values, grouped by the tile size
        if tile == 256:
            assert np.array_equal(tot, ref_tot), (mode, sc)
        else:
            assert np.allclose(tot[:, 1:], ref_tot[:, 1:], rtol=1e-12, atol=0), (mode, sc)
            assert np.allclose(tot[:, 0], ref_tot[:, 0], rtol=0, atol=1e-14), (mode, sc)


def test_schedule_rules(H):
    with pytest.raises(H.HLBMError):
        H.HLBMBatch(ITEMS, "f32", tile=1024)
    with pytest.raises(H.HLBMError):
        H.HLBMBatch(ITEMS, "f32", tile=100)
    b = H.HLBMBatch(ITEMS, "f32", tile=512)
    try:
        sc = b.schedule()
        assert sc == {"tile": 512, "blocks_per_cu": 1, "max_blocks_per_cu": sc["max_blocks_per_cu"], "chunk": 2}
        with pytest.raises(H.HLBMError):
            b.set_schedule(sc["max_blocks_per_cu"] + 1, 0)
        with pytest.raises(H.HLBMError):
            b.set_schedule(0, 65)
        with pytest.raises(H.HLBMError):
            b.set_schedule(-1, 0)
        assert b.schedule() == sc                        # rejected calls change nothing
    finally:
        b.close()


@pytest.mark.parametrize("mode", ["graph", "graph_persistent"])
def test_graph_relaunch_and_odd_even_steps(H, mode):
    """Graph cached per (steps, start buffer, kind): 7 + 7 + 3 steps, then a
    switch of graph kind for 4 more, == 21 per-step."""
    fields = _fields(ITEMS[:2], 5)
    b = H.HLBMBatch(ITEMS[:2], "f32", mode=mode)
    try:
        for k, d in enumerate(fields):
            b.set_porosity(k, d)
        for n in (7, 7, 3):
            b.step(n)
        b.set_mode("graph_persistent" if mode == "graph" else "graph")
        b.step(4)
        b.sync()
        assert b.step_count == 21
        st = b.get_state()[0].cpu().numpy()
    finally:
        b.close()
    st2, _, _ = _run_batch(H, ITEMS[:2], fields, 21, "per_step")
    assert np.array_equal(st, st2)


def test_batch_item_vs_oracle(H):
    it = dict(shape=(32, 32, 32), tau=0.7, force=(1e-6, 0, 0))
    d = inputs.round_to(inputs.batch_item_field(32, 0.5), "f32").astype(np.float32).ravel()
    items = [ITEMS[1], it, ITEMS[2]]
    fields = _fields(items, 9)
    fields[1] = d
    steps = 300
    say("item vs oracle, 300 steps")
    _, mom, _ = _run_batch(H, items, fields, steps, "graph")
    cfg = OracleConfig(q=19, nx=32, ny=32, nz=32, tau=0.7, force=(1e-6, 0, 0))
    g = oracle.run(cfg, d.astype(np.float64), steps, nthreads=NT)
    dr_o, u_o = oracle.observe(cfg, g)
    eu = rel_l2_u(mom[1][1], u_o)
    er = rel_l2_drho(mom[1][0], dr_o, u_o)
    say(f"rel-L2 u {eu:.2e} drho {er:.2e}")
    assert eu <= 1e-5 and er <= 1e-5


def test_unit_cell_workload_full_size(H):
    """256 homogenized unit cells (edges 32..96, phi in [0.1, 0.9], tau in
    [0.55, 1]), body force 1e-6, 2000 steps in one graph launch."""
    import torch
    spec = inputs.batch_items(256, seed=0)
    items = [dict(shape=(e, e, e), tau=t, force=(1e-6, 0, 0)) for e, _, t in spec]
    say("building 256 unit-cell fields")
    fields = [inputs.round_to(inputs.batch_item_field(e, phi), "f32").astype(np.float32).ravel()
              for e, phi, _ in spec]
    from paper_2310_14746_amd import tune
    sched = tune.lookup_batch(items, "f32") or {}      # the schedule bench.py times
    b = H.HLBMBatch(items, "f32", mode="graph", **sched)
    say(f"schedule {b.schedule()}")
    try:
        for k, d in enumerate(fields):
            b.set_porosity(k, d)
        say("2000 steps, one graph launch")
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(b.stream)
        b.step(2000)
        e1.record(b.stream)
        b.sync()
        ms = e0.elapsed_time(e1)
        n, cells = b.info()
        say(f"{cells} cells x 2000 steps in {ms:.0f} ms: {cells * 2000 / ms / 1e3:.0f} MLUPS")
        tot = b.totals()
        k32 = next(k for k, (e, _, _) in enumerate(spec) if e == 32)
        dr, u = (t.cpu().numpy() for t in b.moments(k32))
    finally:
        b.close()
    assert np.isfinite(tot).all()
    cells_k = np.array([e ** 3 for e, _, _ in spec], dtype=float)
    nu = (np.array([t for _, _, t in spec]) - 0.5) / 3.0
    k_darcy = nu * (tot[:, 1] / cells_k) / 1e-6        # k = nu <u_x> / g, rho0 = 1
    assert (k_darcy > 0).all()
    # permeability decreases with solid fraction at fixed edge (monotone trend)
    for e in (32, 64, 96):
        sel = [i for i, (ee, _, _) in enumerate(spec) if ee == e]
        phis = np.array([spec[i][1] for i in sel])
        ks = k_darcy[sel] / nu[sel]
        assert np.corrcoef(phis, ks)[0, 1] > 0.5
    # one 32^3 item against the FP64 oracle at full length
    cfg = OracleConfig(q=19, nx=32, ny=32, nz=32, tau=spec[k32][2], force=(1e-6, 0, 0))
    g = oracle.run(cfg, fields[k32].astype(np.float64), 2000, nthreads=NT)
    dr_o, u_o = oracle.observe(cfg, g)
    eu, er = rel_l2_u(u, u_o), rel_l2_drho(dr, dr_o, u_o)
    say(f"item {k32} (32^3) vs oracle after 2000 steps: u {eu:.2e} drho {er:.2e}")
    assert eu <= 1e-5 and er <= 1e-5


@pytest.mark.parametrize("storage", ["f64", "f16s", "bf16s"])
def test_storage_forms_match_single_contexts(H, storage):
    """FP64 and 16-bit batches: every mode gives the bits of a single context
    of the same storage (graph with the default schedule and with 64-cell
    tiles, persistent, per step)."""
    items = ITEMS[:3]
    fields = _fields(items, 13)
    steps = 17
    scale = 2.0 ** 16 if storage != "f64" else 1.0
    dt = np.float64 if storage == "f64" else np.float16
    refs = []
    for it, d in zip(items, fields):
        sim = H.HLBM(19, storage, it["shape"], tau=it["tau"], force=it["force"], store_scale=scale)
        try:
            sim.set_porosity(d.astype(dt))
            sim.step(steps)
            refs.append(sim.get_state()[0].cpu().numpy())
        finally:
            sim.close()
    for mode, tile in (("graph", 0), ("graph", 64), ("graph_persistent", 0), ("graph_persistent", 64),
                       ("persistent", 0), ("per_step", 0)):
        say(f"{storage} batch, mode {mode}, tile {tile or 'default'}")
        b = H.HLBMBatch(items, storage, store_scale=scale, mode=mode, tile=tile)
        try:
            for k, d in enumerate(fields):
                b.set_porosity(k, d.astype(dt))
            b.step(steps)
            b.sync()
            st = b.get_state()[0].cpu().numpy()
        finally:
            b.close()
        # the packed state: population row i spans all items, item k at its base
        elem = 8 if storage == "f64" else 2
        cells = [int(np.prod(it["shape"])) for it in items]
        ntot = sum(cells)
        packed = st.view(np.uint8).reshape(19, ntot * elem)
        base = 0
        for k, n in enumerate(cells):
            single = refs[k].view(np.uint8).reshape(19, n * elem)
            assert np.array_equal(packed[:, base * elem:(base + n) * elem], single), (mode, tile, k)
            base += n


def test_barrier_bound_error_path(H):
    """A barrier bound of 0 polls makes the persistent kernel's first grid
    barrier fail: every block leaves, the call that syncs reports EDEVICE, and
    after a reset the batch runs again and matches one launch per step."""
    fields = _fields(ITEMS, 17)
    ref, _, _ = _run_batch(H, ITEMS, fields, 9, "per_step")
    for mode in ("persistent", "graph_persistent"):
        say(f"barrier bound 0, mode {mode}")
        b = H.HLBMBatch(ITEMS, "f32", mode=mode)
        try:
            for k, d in enumerate(fields):
                b.set_porosity(k, d)
            b.set_barrier_limit(0)
            b.step(5)
            with pytest.raises(H.HLBMError) as ei:
                b.sync()
            assert ei.value.code == H.EDEVICE and "barrier" in str(ei.value)
            with pytest.raises(H.HLBMError):
                b.set_barrier_limit(-1)
            b.set_barrier_limit(1 << 20)
            b.reset()
            b.step(9)
            b.sync()
            assert np.array_equal(b.get_state()[0].cpu().numpy(), ref)
        finally:
            b.close()


@pytest.mark.parametrize("pad", [256, 8448])
def test_padded_batch_rows_bitwise(H, pad):
    """Padding the packed population rows (items[0].row_pad_bytes) changes
    only where the rows sit: state, totals and per-item moments equal the
    dense-row run bit for bit in every launch mode."""
    fields = _fields(ITEMS, 12)
    steps = 17
    ref, ref_mom, ref_tot = _run_batch(H, ITEMS, fields, steps, "per_step")
    for mode in ("graph", "graph_persistent", "persistent", "per_step"):
        b = H.HLBMBatch(ITEMS, "f32", mode=mode, row_pad=pad)
        try:
            for k, d in enumerate(fields):
                b.set_porosity(k, d)
            b.step(steps)
            b.sync()
            st = b.get_state()[0].cpu().numpy()
            tot = b.totals()
            mom = [tuple(x.cpu().numpy() for x in b.moments(k)) for k in range(len(ITEMS))]
        finally:
            b.close()
        say(f"row pad {pad}, mode {mode}")
        assert np.array_equal(st, ref) and np.array_equal(tot, ref_tot), mode
        for k in range(len(ITEMS)):
            assert np.array_equal(mom[k][0], ref_mom[k][0]) and np.array_equal(mom[k][1], ref_mom[k][1]), (mode, k)


def _masks(items, seed):
    """Random obstacles (about 15% of the cells solid) for every item."""
    out = []
    for k, it in enumerate(items):
        n = int(np.prod(it["shape"]))
        out.append((np.random.default_rng(seed + k).random(n) < 0.15).astype(np.uint8))
    return out


def test_masked_items_match_single_contexts(H):
    """Resolved obstacles per item: an item with a mask evolves bit for bit as
    a single context with the same mask (hlbm_set_solid_mask), an item without
    one as the plain single context, in every launch mode; moments and totals
    follow; removing the masks gives the unmasked batch back."""
    items = ITEMS
    fields = _fields(items, 21)
    masks = _masks(items, 30)
    masked = {0, 2}      # items 1 and 3 stay free of obstacles
    steps = 19
    refs, ref_mom = [], []
    for k, (it, d) in enumerate(zip(items, fields)):
        sim = H.HLBM(19, "f32", it["shape"], tau=it["tau"], force=it["force"])
        try:
            sim.set_porosity(d)
            if k in masked:
                sim.set_solid_mask(masks[k])
            sim.step(steps)
            refs.append(sim.state_f64())
            dr, u = sim.moments("f64")
            ref_mom.append((dr.cpu().numpy(), u.cpu().numpy()))
        finally:
            sim.close()
    for mode in ("graph", "graph_persistent", "persistent", "per_step"):
        say(f"masked items {sorted(masked)}, mode {mode}")
        b = H.HLBMBatch(items, "f32", mode=mode)
        try:
            for k, d in enumerate(fields):
                b.set_porosity(k, d)
                if k in masked:
                    b.set_solid_mask(k, masks[k])
            b.step(steps)
            b.sync()
            st = b.get_state()[0].cpu().numpy().view(np.float32).reshape(19, -1)
            mom = [tuple(x.cpu().numpy() for x in b.moments(k)) for k in range(len(items))]
            tot = b.totals()
        finally:
            b.close()
        base = 0
        for k, it in enumerate(items):
            n = int(np.prod(it["shape"]))
            assert np.array_equal(st[:, base:base + n].astype(np.float64), refs[k]), (mode, k)
            assert np.array_equal(mom[k][0], ref_mom[k][0]) and np.array_equal(mom[k][1], ref_mom[k][1]), (mode, k)
            if k in masked:
                solid = masks[k].reshape(mom[k][0].shape) != 0
                assert (mom[k][0][solid] == 0).all() and (mom[k][1][:, solid] == 0).all()
            # totals: sums over fluid cells of drho and rho u
            dr, u = mom[k]
            want = [dr.sum()] + [((1.0 + dr) * u[a]).sum() for a in range(3)]
            assert np.allclose(tot[k], want, rtol=1e-9, atol=1e-15), (mode, k)
            base += n
    # masks removed: the plain batch again
    ref_plain, _, _ = _run_batch(H, items, fields, steps, "per_step")
    b = H.HLBMBatch(items, "f32", mode="graph")
    try:
        for k, d in enumerate(fields):
            b.set_porosity(k, d)
            b.set_solid_mask(k, masks[k])
        for k in range(len(items)):
            b.set_solid_mask(k, None)
        b.step(steps)
        b.sync()
        assert np.array_equal(b.get_state()[0].cpu().numpy(), ref_plain)
    finally:
        b.close()


def test_masked_sphere_item_vs_oracle(H):
    """A resolved sphere in a periodic 32^3 unit cell, inside a batch, against
    the FP64 oracle's masked run."""
    e, tau = 32, 0.8
    r = inputs.radius_for_porosity(e, 0.6)
    mask = (inputs.sphere_indicator(e, r) > 0.5).astype(np.uint8).ravel()
    it = dict(shape=(e, e, e), tau=tau, force=(1e-6, 0, 0))
    items = [ITEMS[2], it]
    fields = _fields(items, 4)
    fields[1] = np.zeros(e ** 3, dtype=np.float32)
    steps = 300
    say("masked sphere item vs oracle, 300 steps")
    b = H.HLBMBatch(items, "f32", mode="graph")
    try:
        for k, d in enumerate(fields):
            b.set_porosity(k, d)
        b.set_solid_mask(1, mask)
        b.step(steps)
        dr, u = (x.cpu().numpy() for x in b.moments(1))
    finally:
        b.close()
    cfg = OracleConfig(q=19, nx=e, ny=e, nz=e, tau=tau, force=(1e-6, 0, 0))
    g = oracle.run_masked(cfg, mask, np.zeros(e ** 3), steps, nthreads=NT)
    dr_o, u_o = oracle.observe_masked(cfg, mask, g)
    eu = rel_l2_u(u.reshape(3, -1), u_o)
    er = rel_l2_drho(dr.ravel(), dr_o, u_o)
    say(f"rel-L2 u {eu:.2e} drho {er:.2e}")
    assert eu <= 1e-5 and er <= 1e-5
