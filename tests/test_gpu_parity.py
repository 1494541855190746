"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Integer results -- vertex order, gradient, critical sets, arcs and the
(birth, death) simplex pairs of D0, D1, D2 -- must be bit-identical.
"""
import numpy as np
import pytest

import oracle
import synthfields as sf
from tests import helpers as H

SMALL_FIELDS = {
    "noise16_s0": lambda: sf.noise((16, 16, 16), 0),
    "noise16_s1": lambda: sf.noise((16, 16, 16), 1),
    "noise16_s2": lambda: sf.noise((16, 16, 16), 2),
    "noise_aniso": lambda: sf.noise((5, 9, 7), 3),
    "noise_thin": lambda: sf.noise((2, 2, 9), 4),
    "noise_slab": lambda: sf.noise((3, 17, 2), 5),
    "cube2": lambda: np.arange(8, dtype=np.float32)[::-1].reshape(2, 2, 2).copy(),
    "ties": lambda: np.random.default_rng(6).integers(0, 4, size=(9, 8, 7)).astype(np.float32),
    "smooth20": lambda: sf.gaussians((20, 22, 18), 7, k=8, noise_frac=0.01),
    "elevation": lambda: sf.elevation((7, 6, 5)),
    "radial": lambda: sf.radial((17, 17, 17)),
    "neg_zero": lambda: np.where(sf.noise((6, 6, 6), 8) < 0.5, np.float32(-0.0), np.float32(0.0)),
    "infinities": lambda: sf.with_infinities(sf.noise((7, 8, 9), 9), 9),
    "infinities_smooth": lambda: sf.with_infinities(sf.gaussians((12, 10, 11), 10, k=4, noise_frac=0.01), 10, 0.3, 0.1),
}


def _encode_oracle(shape, partner):
    """Oracle partners -> gradient byte codes (test-side encoder, used to
    check the decoder on the CPU)."""
    nz, ny, nx = shape
    V = nx * ny * nz
    G = np.zeros((26, V), dtype=np.uint8)
    for dim in range(4):
        P = partner[dim]
        for t in range(H.NTYPES[dim]):
            ids = np.arange(V) * H.NTYPES[dim] + t
            p = P[ids]
            code = np.zeros(V, dtype=np.uint8)
            code[p == -1] = 0xFF
            code[p == -2] = 0xFE
            ok = p >= 0
            pd, pid = p & 3, p >> 2
            vs_all = H.vertices(shape, dim, ids)
            for sel_up in (True, False):
                sel = ok & ((pd == dim + 1) if sel_up else (pd == dim - 1))
                if not sel.any():
                    continue
                vs = vs_all[sel]
                ws = H.vertices(shape, pd[sel][0] if False else (dim + 1 if sel_up else dim - 1), pid[sel])
                if sel_up:
                    extra = np.array([list(set(w) - set(v))[0] for v, w in zip(vs.tolist(), ws.tolist())])
                    a = H.coords(shape, vs[:, 0])
                    e = H.coords(shape, extra)
                    d = e - a
                    code[sel] = (13 + d[:, 0] + 3 * d[:, 1] + 9 * d[:, 2]).astype(np.uint8)
                else:
                    pos = np.array([[i for i, x in enumerate(v) if x not in set(w)][0]
                                    for v, w in zip(vs.tolist(), ws.tolist())])
                    code[sel] = (0x80 | pos).astype(np.uint8)
            G[H.PLANE_BASE[dim] + t] = code
    return G


def test_gradient_decoder_roundtrip_cpu():
    f = sf.noise((5, 6, 7), 2)
    res = oracle.run(f)
    G = _encode_oracle(res.shape, res.partner)
    dec = H.decode_gradient(res.shape, G)
    for d in range(4):
        assert np.array_equal(dec[d], res.partner[d])


def _gpu_ctx():
    import torch
    from paper_2206_13932_amd import dms
    return torch, dms, dms.Context(0)


def _check_all(name, f, ctx, torch, dms):
    print(f"[parity] case={name} shape={f.shape}", flush=True)
    res = oracle.run(f)
    ft = torch.from_numpy(f).cuda()
    ncrit = ctx.gradient(ft)
    assert ncrit == [len(c) for c in res.crit], name
    rank = ctx.debug(dms.BUF_RANK)
    assert np.array_equal(rank, res.rank), name
    G = ctx.debug(dms.BUF_GRADIENT, np.uint8)
    dec = H.decode_gradient(res.shape, G)
    for d in range(4):
        assert np.array_equal(dec[d], res.partner[d]), (name, d)
    for d in range(4):
        got = ctx.debug(dms.BUF_CRIT0 + d).astype(np.int64)
        assert np.array_equal(got, res.crit[d]), (name, "crit", d)
    d0, d2 = ctx.pairs_d0_d2()
    arcs0 = ctx.debug(dms.BUF_ARCS0).reshape(2, -1).T.astype(np.int64)
    exp0 = res.rank[res.arcs0[:, :2]].astype(np.int64)
    assert np.array_equal(arcs0, exp0), (name, "arcs0")
    assert np.array_equal(d0.cpu().numpy(), res.pairs[0]), (name, "D0")
    exp2 = res.pairs[2][res.pairs[2][:, 1] >= 0]
    assert np.array_equal(d2.cpu().numpy(), exp2), (name, "D2")
    # dual arcs (D2 in 3D, D1 on 2D grids): the ages of the two maxima each
    # saddle reaches, saddles in decreasing order; 0 = virtual maximum, 1 = the
    # highest maximum; the two sides as an unordered pair
    top = res.crit[2 if res.shape[0] == 1 else 3]
    age = {int(t): len(top) - i for i, t in enumerate(top)}
    exp_arcs = np.array([[0 if a < 0 else age[int(a)], 0 if b < 0 else age[int(b)]] for a, b, _ in res.arcs2],
                        dtype=np.int64).reshape(-1, 2)
    got_arcs = ctx.debug(dms.BUF_ARCS2).reshape(2, -1).T.astype(np.int64)
    assert np.array_equal(np.sort(got_arcs, axis=1), np.sort(exp_arcs, axis=1)), (name, "dual arcs")
    d1 = ctx.pairs_d1()
    assert np.array_equal(d1.cpu().numpy(), res.pairs[1]), (name, "D1")
    out = ctx.diagram(ft)
    for d in range(3):
        assert np.array_equal(out[d].cpu().numpy(), res.pairs[d]), (name, "diagram", d)
    return res


@pytest.mark.gpu
@pytest.mark.parametrize("name", sorted(SMALL_FIELDS))
def test_parity_small(name):
    torch, dms, ctx = _gpu_ctx()
    _check_all(name, SMALL_FIELDS[name](), ctx, torch, dms)
    ctx.close()


@pytest.mark.gpu
def test_parity_many_noise_seeds_one_context():
    torch, dms, ctx = _gpu_ctx()
    for seed in range(10, 26):
        f = sf.noise((16, 16, 16), seed)
        res = oracle.run(f)
        out = ctx.diagram(torch.from_numpy(f).cuda())
        for d in range(3):
            assert np.array_equal(out[d].cpu().numpy(), res.pairs[d]), (seed, d)
    ctx.close()


@pytest.mark.gpu
@pytest.mark.parametrize("shape,kind", [((40, 40, 40), "noise"), ((64, 64, 64), "smooth"),
                                        ((33, 47, 61), "smooth")])
def test_parity_multi_tile(shape, kind):
    torch, dms, ctx = _gpu_ctx()
    f = sf.noise(shape, 9) if kind == "noise" else sf.gaussians(shape, 9, k=16, noise_frac=0.01)
    _check_all(f"{kind}{shape}", f, ctx, torch, dms)
    ctx.close()


@pytest.mark.gpu
def test_diagram_values():
    torch, dms, ctx = _gpu_ctx()
    f = sf.gaussians((24, 20, 16), 3, k=6, noise_frac=0.01)
    res = oracle.run(f)
    out = ctx.diagram(torch.from_numpy(f).cuda(), with_values=True)
    fv = f.ravel()
    for d in range(3):
        o = out[d]
        p = o["pairs"].cpu().numpy()
        assert np.array_equal(p, res.pairs[d])
        bv = oracle.simplex_vertices(res.shape, d, p[:, 0])
        exp_b = bv[np.arange(len(bv)), res.rank[bv].argmax(axis=1)]
        assert np.array_equal(o["birth_vertex"].cpu().numpy(), exp_b)
        assert np.array_equal(o["birth_value"].cpu().numpy(), fv[exp_b])
        fin = p[:, 1] >= 0
        dvv = o["death_vertex"].cpu().numpy()
        assert (dvv[~fin] == -1).all()
        assert np.array_equal(o["death_value"].cpu().numpy()[~fin], np.full((~fin).sum(), fv.max(), np.float32))
        if fin.any():
            dv = oracle.simplex_vertices(res.shape, d + 1, p[fin, 1])
            exp_d = dv[np.arange(len(dv)), res.rank[dv].argmax(axis=1)]
            assert np.array_equal(dvv[fin], exp_d)
    ctx.close()


@pytest.mark.gpu
def test_error_paths():
    torch, dms, ctx = _gpu_ctx()
    import ctypes
    f = torch.from_numpy(sf.noise((6, 6, 6), 0)).cuda()
    n0, n2 = ctypes.c_int64(), ctypes.c_int64()
    rc = ctx.lib.dms_pairs_d0_d2(ctx.h, None, 0, ctypes.byref(n0), None, 0, ctypes.byref(n2))
    assert rc == dms.DMS_E_STATE
    g = f.clone()
    g[2, 3, 4] = float("nan")
    with pytest.raises(dms.DmsError) as e:
        ctx.gradient(g)
    assert e.value.code == dms.DMS_E_NAN
    with pytest.raises(dms.DmsError) as e:
        ctx.gradient(torch.zeros((2, 1, 5), device="cuda"))
    assert e.value.code == dms.DMS_E_INVAL
    ctx.gradient(f)
    n1 = ctypes.c_int64()
    rc = ctx.lib.dms_pairs_d1(ctx.h, None, 0, ctypes.byref(n1))
    assert rc == dms.DMS_E_STATE
    n0, n2 = ctypes.c_int64(), ctypes.c_int64()
    buf = torch.empty((1, 2), dtype=torch.int64, device="cuda")
    rc = ctx.lib.dms_pairs_d0_d2(ctx.h, ctypes.c_void_p(buf.data_ptr()), 1, ctypes.byref(n0),
                                 ctypes.c_void_p(buf.data_ptr()), 1, ctypes.byref(n2))
    assert rc == dms.DMS_E_CAPACITY and n0.value > 1
    ctx.close()
    small = dms.Context(0, hbm_budget=1 << 16)
    with pytest.raises(dms.DmsError) as e:
        small.gradient(torch.from_numpy(sf.noise((32, 32, 32), 0)).cuda())
    assert e.value.code == dms.DMS_E_NOMEM
    small.close()


@pytest.mark.gpu
def test_hbm_budget_bounds_every_stage():
    """Budgets doubling from 64 KiB: each diagram either equals the oracle's or
    fails with DMS_E_NOMEM; D1's storage and the generator export count
    against the budget too (some budget runs out inside D1)."""
    import torch
    from paper_2206_13932_amd import dms
    f = sf.noise((32, 32, 32), 12)
    res = oracle.run(f)
    ft = torch.from_numpy(f).cuda()
    messages, ok = [], 0
    for k in range(16, 32):
        print(f"[parity] budget 2^{k}", flush=True)
        ctx = dms.Context(0, hbm_budget=1 << k)
        try:
            out = ctx.diagram(ft)
            for d in range(3):
                assert np.array_equal(out[d].cpu().numpy(), res.pairs[d]), (k, d)
            off, edges = ctx.d1_generators()
            assert off.numel() == int((res.pairs[1][:, 1] >= 0).sum()) + 1
            ok += 1
        except dms.DmsError as e:
            assert e.code == dms.DMS_E_NOMEM, (k, e.code, str(e))
            messages.append(str(e))
        finally:
            ctx.close()
    assert ok > 0 and messages
    assert any("D1" in m or "generators" in m for m in messages), messages


@pytest.mark.gpu
def test_parity_d1_every_deferral_pass():
    """Tiny working heaps (the context's debug option) force columns through
    all D1 passes (LDS heaps of two sizes, then workgroup passes), and every
    cached boundary longer than two entries is added by the full merge; pairs
    must not change, and the cycles published by every kind of pass must be
    valid generators. Those full merges are split into parts of 40 merged
    positions (one cooperative merge per addition, helped by idle workgroups
    of the pass). A second context without the option, used in between,
    keeps the production plan."""
    torch, dms, ctx = _gpu_ctx()
    ctx.set_option(dms.OPT_D1_SMALL_PASSES, 1)
    plain = dms.Context(0)
    longs = coop = 0
    for name, f in [("noise24", sf.noise((24, 24, 24), 3)),
                    ("smooth40", sf.gaussians((40, 36, 32), 4, k=12, noise_frac=0.01))]:
        print(f"[parity] case=d1_small_passes/{name}", flush=True)
        res = oracle.run(f)
        ft = torch.from_numpy(f).cuda()
        out = ctx.diagram(ft)
        st = ctx.debug(dms.BUF_STATS, np.uint64).tolist()
        print(name, "deferrals", st[7], "passes", st[10:20], "full-merge additions", st[41],
              "cooperative merges", st[44], "helped parts", st[45], flush=True)
        assert st[7] > 0
        longs += st[41]
        coop += st[44]
        for d in range(3):
            assert np.array_equal(out[d].cpu().numpy(), res.pairs[d]), (name, d)
        off, edges = ctx.d1_generators()
        d1 = out[1].cpu().numpy()
        fin = d1[d1[:, 1] >= 0]
        status = oracle.bf_check_cycles(res.shape, res.rank, fin, off.cpu().numpy(), edges.cpu().numpy())
        assert (status == 0).all(), (name, np.bincount(status))
        ref = plain.diagram(ft)
        pst = plain.debug(dms.BUF_STATS, np.uint64).tolist()
        assert pst[7] < st[7], (name, pst[7], st[7])  # the option stays with its context
        for d in range(3):
            assert np.array_equal(ref[d].cpu().numpy(), res.pairs[d]), (name, "plain", d)
    assert longs > 0 and coop > 0
    with pytest.raises(dms.DmsError):
        ctx.set_option(99, 1)
    ctx.close()
    plain.close()


@pytest.mark.gpu
@pytest.mark.skip(reason="not yet run on a GPU: the D1 restart it drives is a suspect of the quarantined "
                         "512^3 noise fault, so its first run is a run of its own")
def test_parity_d1_restart():
    """A publication heap smaller than the cached boundaries need (the
    context's debug option) makes D1 overflow it, grow it and run again from
    its first pass; the pairs must not change. The heap starts at half of what
    a plain run publishes, so that it doubles once or twice."""
    torch, dms, ctx = _gpu_ctx()
    plain = dms.Context(0)
    for name, f in [("noise40", sf.noise((40, 44, 48), 11)),
                    ("smooth48", sf.gaussians((48, 48, 48), 5, k=12, noise_frac=0.02))]:
        print(f"[parity] case=d1_restart/{name}", flush=True)
        res = oracle.run(f)
        ft = torch.from_numpy(f).cuda()
        ref = plain.diagram(ft)
        published = int(plain.debug(dms.BUF_STATS, np.uint64)[8])
        assert published > 256, (name, published)
        ctx.set_option(dms.OPT_D1_HEAP_KEYS, published // 2)
        out = ctx.diagram(ft)
        st = ctx.debug(dms.BUF_STATS, np.uint64).tolist()
        print(name, "published", published, "restarts", st[9], flush=True)
        assert 1 <= st[9] <= 3, (name, st[9])
        for d in range(3):
            assert np.array_equal(out[d].cpu().numpy(), res.pairs[d]), (name, d)
            assert np.array_equal(ref[d].cpu().numpy(), res.pairs[d]), (name, "plain", d)
        off, edges = ctx.d1_generators()
        d1 = out[1].cpu().numpy()
        fin = d1[d1[:, 1] >= 0]
        status = oracle.bf_check_cycles(res.shape, res.rank, fin, off.cpu().numpy(), edges.cpu().numpy())
        assert (status == 0).all(), (name, np.bincount(status))
    with pytest.raises(dms.DmsError):
        ctx.set_option(dms.OPT_D1_HEAP_KEYS, -1)
    ctx.close()
    plain.close()


@pytest.mark.gpu
@pytest.mark.parametrize("variant", ["no_sandwich", "no_cache", "neither"])
def test_parity_d1_ablation_variants(variant):
    """PairCriticalSimplices without the sandwich (every 2-saddle a column,
    no 1-saddle set aside) and/or without boundary caching (an earlier owner's
    2-saddle boundary re-reduced) gives the same pairs as the oracle: with the
    virtual maximum (and without it for the variant without caching; the one
    without the sandwich is refused there), and through every D1 pass (small
    capacities)."""
    torch, dms, ctx = _gpu_ctx()
    opts = {"no_sandwich": [dms.OPT_D1_NO_SANDWICH], "no_cache": [dms.OPT_D1_NO_CACHE],
            "neither": [dms.OPT_D1_NO_SANDWICH, dms.OPT_D1_NO_CACHE]}[variant]
    for o in opts:
        ctx.set_option(o, 1)
    cases = [("noise16_s0", SMALL_FIELDS["noise16_s0"](), True), ("smooth20", SMALL_FIELDS["smooth20"](), True),
             ("ties", SMALL_FIELDS["ties"](), True), ("noise_aniso", SMALL_FIELDS["noise_aniso"](), True),
             ("noise16_s1 off", SMALL_FIELDS["noise16_s1"](), False), ("infinities off", SMALL_FIELDS["infinities"](), False)]
    for small in (False, True):
        ctx.set_option(dms.OPT_D1_SMALL_PASSES, 1 if small else 0)
        for name, f, vmax in cases:
            print(f"[ablation] variant={variant} case={name} small={small}", flush=True)
            ft = torch.from_numpy(f).cuda()
            if not vmax and variant != "no_cache":
                # without the virtual maximum the sandwich is part of the mode's
                # definition: the ablation is refused
                with pytest.raises(dms.DmsError):
                    ctx.diagram(ft, flags=0)
                continue
            res = oracle.run(f, virtual_max=vmax)
            out = ctx.diagram(ft, flags=dms.DMS_VIRTUAL_MAX if vmax else 0)
            for d in range(3):
                assert np.array_equal(out[d].cpu().numpy(), res.pairs[d]), (variant, name, small, d)
    st = ctx.debug(dms.BUF_STATS, np.uint64).tolist()
    assert st[4] > 0  # the last diagram ran D1 steps
    ctx.close()


# ---- without the virtual maximum on the domain boundary (Sec. 5.2, App. A) ----

OFF_FIELDS = dict(SMALL_FIELDS)
OFF_FIELDS.update({
    "noise40": lambda: sf.noise((40, 40, 40), 11),
    "smooth_tiles": lambda: sf.gaussians((33, 47, 61), 12, k=10, noise_frac=0.01),
    "noise_2d": lambda: sf.noise((1, 64, 53), 13),
    "smooth_2d": lambda: sf.gaussians((1, 96, 80), 14, k=8, noise_frac=0.01),
    "radial_2d": lambda: sf.radial((1, 17, 17)),
})


@pytest.mark.gpu
@pytest.mark.parametrize("name", sorted(OFF_FIELDS))
def test_parity_virtual_max_off(name):
    """flags = 0: the dual union-find has no outside node; D0, D1, D2 with
    their infinite classes bit for bit against the oracle in the same mode,
    through dms_diagram and through the staged calls."""
    torch, dms, ctx = _gpu_ctx()
    f = OFF_FIELDS[name]()
    print(f"[parity-off] case={name} shape={f.shape}", flush=True)
    res = oracle.run(f, virtual_max=False)
    ft = torch.from_numpy(f).cuda()
    out = ctx.diagram(ft, flags=0)
    for d in (0, 2, 1):  # D2 first: it decides which 2-saddles D1 takes
        assert np.array_equal(out[d].cpu().numpy(), res.pairs[d]), (name, d)
    ctx.gradient(ft, flags=0)
    d0, d2 = ctx.pairs_d0_d2()
    assert np.array_equal(d0.cpu().numpy(), res.pairs[0]), name
    if f.shape[0] > 1:  # the staged D2 call reports the finite pairs (the infinite ones come after D1)
        assert np.array_equal(d2.cpu().numpy(), res.pairs[2][res.pairs[2][:, 1] >= 0]), name
        d1 = ctx.pairs_d1()
        assert np.array_equal(d1.cpu().numpy(), res.pairs[1]), name
    # the mode belongs to the call: the default comes back with the flag
    on = ctx.diagram(ft)
    ref = oracle.run(f)
    for d in range(3):
        assert np.array_equal(on[d].cpu().numpy(), ref.pairs[d]), (name, "on", d)
    ctx.close()


@pytest.mark.gpu
def test_virtual_max_off_is_refused_in_batches_and_unknown_flags():
    torch, dms, ctx = _gpu_ctx()
    f = torch.from_numpy(sf.noise((8, 9, 10), 0)).cuda()
    with pytest.raises(dms.DmsError):
        ctx.diagram_batch([f], flags=0)
    with pytest.raises(dms.DmsError):
        ctx.diagram(f, flags=4)
    assert np.array_equal(ctx.diagram(f)[0].cpu().numpy(), oracle.run(f.cpu().numpy()).pairs[0])
    ctx.close()
