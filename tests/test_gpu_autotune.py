"""The autotuners: the training-step tilings picked by ann_autotune_train
give the gradients of the built-in tilings (up to the FP32 summation order
of a different split along the batch), on the single network and the
per-species ensemble; both tuners store their results in the file named by
CHEM_AUTOTUNE_CACHE and take them from there on the next call."""
import os
import sys
import tempfile

import numpy as np
import pytest

import chemgen
import oracle
from gpu_util import need_gpu, to_dev

pytestmark = pytest.mark.gpu

HID = (1600, 800, 400)


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    return need_gpu()


@pytest.fixture(scope="module")
def data():
    mech = chemgen.make_mechanism("ch4")
    om = oracle.OracleMech(mech)
    T, p, Y0 = chemgen.make_states(mech, "ch4", N=8192, seed=5151)
    o = oracle.chem_step(om, 1e-5, T, p, Y0)
    return mech, dict(T=T, p=p, Y0=Y0, Y1=o["Y"])


def _grads(m, K, members):
    sh = [(HID[0], K + 2), (HID[1], HID[0]), (HID[2], HID[1]), ((1 if members > 1 else K), HID[2])]
    return [m.get_grad(4 * g + l, sh[l]) for g in range(members) for l in range(4)]


@pytest.mark.parametrize("members", [1, 30])
def test_tuned_training_step_gives_the_same_gradients(dev, data, members, monkeypatch):
    import torch
    import paper_2312_05800_amd as P
    mech, d = data
    K = mech.K
    monkeypatch.delenv("CHEM_AUTOTUNE_CACHE", raising=False)
    _say(f"[autotune train] members={members}")
    B = 8192
    dv = {k: to_dev(v, dev) for k, v in d.items()}
    loss = torch.zeros(1, dtype=torch.float32, device=dev)
    m = P.AnnModel(K + 2, K, HID, seed=3, members=members)
    m.fit_norm(dv["T"], dv["p"], dv["Y0"], dv["Y1"], 0.1, 1e-5)
    m.train_step(dv["T"], dv["p"], dv["Y0"], dv["Y1"], loss, lr=0.0)
    torch.cuda.synchronize()
    g0 = _grads(m, K, members)
    l0 = loss.item()
    t = m.autotune_train(B)
    _say(f"  products: built-in {t['products_ms_default']:.3f} ms, "
         f"tuned {t['products_ms_tuned']:.3f} ms")
    assert 0 < t["products_ms_tuned"] <= t["products_ms_default"]
    m.train_step(dv["T"], dv["p"], dv["Y0"], dv["Y1"], loss, lr=0.0)
    torch.cuda.synchronize()
    assert loss.item() == l0  # the forward's rounding does not depend on the tiling's split
    for (a, b), (c, e) in zip(_grads(m, K, members), g0):
        for x, y in ((a, c), (b, e)):
            rel = np.linalg.norm(x - y) / max(np.linalg.norm(y), 1e-30)
            assert rel <= 1e-5, rel


def test_tuning_cache_round_trip(dev, data, monkeypatch):
    import torch
    import paper_2312_05800_amd as P
    mech, d = data
    K = mech.K
    with tempfile.TemporaryDirectory() as tmp:
        path = os.path.join(tmp, "tune.txt")
        monkeypatch.setenv("CHEM_AUTOTUNE_CACHE", path)
        m = P.AnnModel(K + 2, K, HID, seed=4)
        t1 = m.autotune_train(2048)
        m2 = P.AnnModel(K + 2, K, HID, seed=5)
        t2 = m2.autotune_train(2048)  # from the file: the same numbers, no timing
        assert t1 == t2
        gm = P.Mechanism(mech)
        T, p, Y = (to_dev(a[..., :4096], dev) for a in (d["T"], d["p"], d["Y0"]))
        s1 = P.chem_autotune(gm, 1e-5, T, p, Y.contiguous())
        gm2 = P.Mechanism(mech)
        s2 = P.chem_autotune(gm2, 1e-5, T, p, Y.contiguous())
        assert s1 == s2
        lines = open(path).read().splitlines()
        _say(f"  cache: {lines}")
        assert len(lines) == 2 and lines[0].startswith("ann_train ") and \
            lines[1].startswith("chem_step ")
        torch.cuda.synchronize()
