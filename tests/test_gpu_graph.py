"""Captured steps (HIP graphs) and the integrator's launch autotuner, through
the C ABI: every replay of a captured step equals the eager call bit for bit
(the same kernels on the same inputs; per-cell results do not depend on the
order in which the persistent queue hands out cells), and the autotuned
launch shape keeps the integrator's parity with the oracle."""
import sys

import numpy as np
import pytest

import chemgen
import oracle
from oracle import ann as oann
from gpu_util import need_gpu, to_dev, compare_state

pytestmark = pytest.mark.gpu

HID = (1600, 800, 400)


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    return need_gpu()


@pytest.fixture(scope="module")
def mech():
    return chemgen.make_mechanism("ch4")


def _norm(mech):
    om = oracle.OracleMech(mech)
    T, p, Y0 = chemgen.make_states(mech, "ch4", N=512, seed=505)
    o = oracle.chem_step(om, 1e-5, T, p, Y0)
    feat = oann.features(T, p, Y0, 0.1)
    tgt = oann.targets(Y0, o["Y"], 0.1)
    mi, si = oann.zstats(feat)
    mo, so = oann.zstats(tgt)
    return dict(mu_in=mi, sd_in=si, lo=feat.min(axis=1), hi=feat.max(axis=1), mu_out=mo,
                sd_out=so), (T, p, Y0, o["Y"])


def test_chem_step_graph_replays(dev, mech):
    import torch
    import paper_2312_05800_amd as P
    _say("[graph] chem_step")
    K = mech.K
    gm = P.Mechanism(mech)
    N = 600
    T, p, Y = chemgen.make_states(mech, "ch4", N=N, seed=811)
    pd = to_dev(p, dev)
    Te, Ye = to_dev(T, dev), to_dev(Y, dev)
    se = torch.zeros((3, N), dtype=torch.int32, device=dev)
    P.chem_step(gm, 1e-5, Te, pd, Ye, stats=se)
    torch.cuda.synchronize()
    Tg, Yg = to_dev(T, dev), to_dev(Y, dev)
    sg = torch.zeros((3, N), dtype=torch.int32, device=dev)
    g = P.chem_step_graph(gm, 1e-5, Tg, pd, Yg, stats=sg)
    Tx, Yx = to_dev(T, dev), to_dev(Y, dev)
    for rep in range(3):
        Tg.copy_(to_dev(T, dev))
        Yg.copy_(to_dev(Y, dev))
        sg.zero_()
        torch.cuda.synchronize()
        g.launch()
        torch.cuda.synchronize()
        assert torch.equal(Tg, Te) and torch.equal(Yg, Ye) and torch.equal(sg, se), rep
        # eager work between replays
        P.chem_step(gm, 1e-5, Tx, pd, Yx)
        torch.cuda.synchronize()
    del g
    oc = oracle.chem_step(oracle.OracleMech(mech), 1e-5, T, p, Y)
    res = compare_state(Tg.cpu().numpy(), Yg.cpu().numpy(), oc["T"], oc["Y"])
    assert res["ok"], res


def test_ann_step_graph_replays_and_follows_training(dev, mech):
    import torch
    import paper_2312_05800_amd as P
    _say("[graph] ann_step")
    K = mech.K
    nm, (Tt, pt, Y0t, Y1t) = _norm(mech)
    params = oann.init_params([K + 2, *HID, K], seed=21)
    params[3] = (params[3][0] * 0.02, params[3][1] * 0.02)
    m = P.AnnModel(K + 2, K, HID, seed=1)
    for l, (W, b) in enumerate(params):
        m.set_layer(l, W, b)
    m.set_norm(0.1, 1e-5, nm["mu_in"], nm["sd_in"], nm["lo"], nm["hi"], nm["mu_out"],
               nm["sd_out"])
    gm = P.Mechanism(mech)
    N = 3001
    T, p, Y = chemgen.make_states(mech, "ch4", N=N, seed=812)
    pd = to_dev(p, dev)

    def eager(dt):
        Te, Ye = to_dev(T, dev), to_dev(Y, dev)
        RR = torch.zeros((K, N), dtype=torch.float64, device=dev)
        fl = torch.zeros(N, dtype=torch.uint8, device=dev)
        nf = torch.zeros(1, dtype=torch.int64, device=dev)
        m.step(gm, dt, Te, pd, Ye, RR=RR, flags=fl, n_fallback=nf)
        torch.cuda.synchronize()
        return Te, Ye, RR, fl, nf

    for dt in (1e-5, 2e-6):  # the trained dt, and every cell falling back
        ref = eager(dt)
        Tg, Yg = to_dev(T, dev), to_dev(Y, dev)
        RR = torch.zeros((K, N), dtype=torch.float64, device=dev)
        fl = torch.zeros(N, dtype=torch.uint8, device=dev)
        nf = torch.zeros(1, dtype=torch.int64, device=dev)
        g = m.step_graph(gm, dt, Tg, pd, Yg, RR=RR, flags=fl, n_fallback=nf)
        for rep in range(3):
            Tg.copy_(to_dev(T, dev))
            Yg.copy_(to_dev(Y, dev))
            torch.cuda.synchronize()
            g.launch()
            torch.cuda.synchronize()
            for a, b in zip((Tg, Yg, RR, fl, nf), ref):
                assert torch.equal(a, b), (dt, rep)
            eager(dt)  # eager work between replays
        _say(f"  dt={dt:g}: {int(nf.item())} of {N} cells fell back, 3 replays equal")
        if dt == 2e-6:
            assert int(nf.item()) == N
            # the workspace is held by the graph: a larger step is refused
            T2, p2, Y2 = chemgen.make_states(mech, "ch4", N=N + 64, seed=813)
            with pytest.raises(P.ChemError):
                m.step(gm, 1e-5, to_dev(T2, dev), to_dev(p2, dev), to_dev(Y2, dev))
            del g
            m.step(gm, 1e-5, to_dev(T2, dev), to_dev(p2, dev), to_dev(Y2, dev))
            torch.cuda.synchronize()
        else:
            # a training step between replays: the graph uses the new weights
            loss = torch.zeros(1, dtype=torch.float32, device=dev)
            B = 512
            m.train_step(to_dev(Tt, dev), to_dev(pt, dev), to_dev(Y0t, dev), to_dev(Y1t, dev),
                         loss, B=B, lr=1e-3)
            torch.cuda.synchronize()
            ref2 = eager(dt)
            assert not torch.equal(ref2[1], ref[1])
            Tg.copy_(to_dev(T, dev))
            Yg.copy_(to_dev(Y, dev))
            torch.cuda.synchronize()
            g.launch()
            torch.cuda.synchronize()
            for a, b in zip((Tg, Yg, RR, fl, nf), ref2):
                assert torch.equal(a, b)
            del g


def test_autotune_keeps_parity(dev, mech):
    import torch
    import paper_2312_05800_amd as P
    _say("[autotune] integrator launch shape")
    K = mech.K
    gm = P.Mechanism(mech)
    d0 = P.chem_get_tuning(gm)
    assert d0["lanes_per_cell"] == 32 and d0["waves_per_cu"] >= 1
    T, p, Y = chemgen.make_states(mech, "ch4", N=4096, seed=814)
    Td, pd, Yd = to_dev(T, dev), to_dev(p, dev), to_dev(Y, dev)
    best = P.chem_autotune(gm, 1e-5, Td, pd, Yd)
    torch.cuda.synchronize()
    _say(f"  default {d0}, tuned {best}")
    assert best["lanes_per_cell"] in (32, 64) and 1 <= best["waves_per_cu"] <= 32
    assert best["cells_per_s"] > 0
    assert torch.equal(Td, to_dev(T, dev)) and torch.equal(Yd, to_dev(Y, dev))
    got = P.chem_get_tuning(gm)
    assert (got["lanes_per_cell"], got["waves_per_cu"]) == (best["lanes_per_cell"],
                                                            best["waves_per_cu"])
    # every shape the tuner may pick integrates like the oracle
    om = oracle.OracleMech(mech)
    T2, p2, Y2 = chemgen.make_states(mech, "ch4", N=256, seed=815)
    oc = oracle.chem_step(om, 1e-5, T2, p2, Y2)
    for lanes, waves in ((best["lanes_per_cell"], best["waves_per_cu"]), (64, 3), (32, 2)):
        P.chem_set_tuning(gm, lanes, waves)
        Tg, Yg = to_dev(T2, dev), to_dev(Y2, dev)
        P.chem_step(gm, 1e-5, Tg, to_dev(p2, dev), Yg)
        torch.cuda.synchronize()
        res = compare_state(Tg.cpu().numpy(), Yg.cpu().numpy(), oc["T"], oc["Y"])
        assert res["ok"], (lanes, waves, res)
    with pytest.raises(P.ChemError):
        P.chem_set_tuning(gm, 16, 0)  # 16 lanes cannot hold K + 1 = 31 components
    P.chem_set_tuning(gm, default=True)
    assert P.chem_get_tuning(gm) == d0


def test_step_sets_graph_replays(dev, mech):
    """Uneven sets captured once: the graph keeps its own copy of the set
    table, so an eager chem_step_sets on other sets between replays does not
    change what it integrates; every replay equals the eager call."""
    import torch
    import paper_2312_05800_amd as P
    _say("[graph] chem_step_sets")
    gm = P.Mechanism(mech)
    sizes, dts = [0, 5, 120, 700], [1e-6, 1e-5, 3e-7, 2e-6]
    host = []
    for i, (nc, dt) in enumerate(zip(sizes, dts)):
        T, p, Y = chemgen.make_states(mech, dict(fuel="CH4", phi=(0.5, 1.3),
                                                 T=("uniform", 300.0, 2500.0), N=nc),
                                      seed=900 + i)
        host.append((T, p, Y, dt))

    def fresh():
        return [dict(dt=dt, T=to_dev(T, dev), p=to_dev(p, dev), Y=to_dev(Y, dev),
                     RR=torch.zeros((mech.K, T.size), dtype=torch.float64, device=dev),
                     stats=torch.zeros((3, T.size), dtype=torch.int32, device=dev))
                for T, p, Y, dt in host]

    ref = fresh()
    P.chem_step_sets(gm, ref)
    torch.cuda.synchronize()
    sets = fresh()
    g = P.chem_step_sets_graph(gm, sets)
    other = fresh()[1:3]
    for rep in range(3):
        for d, (T, p, Y, dt) in zip(sets, host):
            d["T"].copy_(to_dev(T, dev))
            d["Y"].copy_(to_dev(Y, dev))
        torch.cuda.synchronize()
        g.launch()
        torch.cuda.synchronize()
        for d, r in zip(sets, ref):
            for k in ("T", "Y", "RR", "stats"):
                assert torch.equal(d[k], r[k]), (rep, k)
        P.chem_step_sets(gm, other)  # eager work on another table
        torch.cuda.synchronize()
    del g
