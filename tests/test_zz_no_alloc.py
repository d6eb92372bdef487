"""ann_step_noalloc (workspace in the library's static device array) against
ann_step (growable workspace) through the C ABI: the same kernels run on the
same inputs, so every output must be identical bit for bit -- T, Y, RR,
flags and the fallback count -- on two calls in a row, the second with fewer
cells, with some cells falling back to the FP64 integrator, and again with
the FP8 hidden layers.  A batch beyond the array's capacity is rejected on
the host."""
import sys

import numpy as np
import pytest

import chemgen
import oracle
from oracle import ann as oann
from gpu_util import need_gpu, to_dev

pytestmark = pytest.mark.gpu

HID = (1600, 800, 400)


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def setup():
    import paper_2312_05800_amd as P
    dev = need_gpu()
    mech = chemgen.make_mechanism("ch4")
    om = oracle.OracleMech(mech)
    K = mech.K
    T, p, Y0 = chemgen.make_states(mech, "ch4", N=1024, seed=505)
    Y1 = oracle.chem_step(om, 1e-5, T, p, Y0)["Y"]
    feat = oann.features(T, p, Y0, 0.1)
    mi, si = oann.zstats(feat)
    mo, so = oann.zstats(oann.targets(Y0, Y1, 0.1))
    params = oann.init_params([K + 2, *HID, K], seed=23)
    # output weights scaled by 20: a good share of the cells exceed the
    # element-residual tolerance and take the FP64 fallback
    params[3] = (params[3][0] * 20.0, params[3][1])
    m = P.AnnModel(K + 2, K, HID, seed=1)
    for layer, (W, b) in enumerate(params):
        m.set_layer(layer, W, b)
    m.set_norm(0.1, 1e-5, mi, si, feat.min(axis=1), feat.max(axis=1), mo, so)
    return dict(P=P, dev=dev, mech=mech, gm=P.Mechanism(mech), m=m, K=K)


def _both(s, N, seed):
    """One ann_step and one ann_step_noalloc on copies of the same states."""
    import torch
    P, dev, mech, gm, m, K = (s[k] for k in ("P", "dev", "mech", "gm", "m", "K"))
    T, p, Y = chemgen.make_states(mech, "ch4", N=N, seed=seed)
    out = []
    for noalloc in (False, True):
        Td, pd, Yd = to_dev(T, dev), to_dev(p, dev), to_dev(Y, dev)
        RR = torch.zeros((K, N), dtype=torch.float64, device=dev)
        flags = torch.zeros(N, dtype=torch.uint8, device=dev)
        nfb = torch.zeros(1, dtype=torch.int64, device=dev)
        m.step(gm, 1e-5, Td, pd, Yd, RR=RR, flags=flags, n_fallback=nfb, noalloc=noalloc)
        torch.cuda.synchronize()
        out.append(dict(T=Td.cpu().numpy(), Y=Yd.cpu().numpy(), RR=RR.cpu().numpy(),
                        flags=flags.cpu().numpy(), nfb=int(nfb.item())))
    return out


def _same(a, b, label):
    nfl = int(np.count_nonzero(a["flags"]))
    _say(f"  {label}: fallback cells {a['nfb']} (flagged {nfl}) vs {b['nfb']}")
    assert a["nfb"] == b["nfb"] and a["nfb"] == nfl
    for k in ("T", "Y", "RR", "flags"):
        assert np.array_equal(a[k], b[k]), k


def test_noalloc_equals_ann_step(setup):
    _say("[ann_step_noalloc vs ann_step, BF16]")
    for N, seed in ((3001, 71), (777, 72)):
        a, b = _both(setup, N, seed)
        assert 0 < a["nfb"] < N  # both the network and the fallback are exercised
        _same(a, b, f"{N} cells")


def test_noalloc_fp8_equals_ann_step(setup):
    import torch
    _say("[ann_step_noalloc vs ann_step, FP8 hidden layers]")
    s = setup
    T, p, Y = chemgen.make_states(s["mech"], "ch4", N=4096, seed=73)
    s["m"].quantize_fp8(to_dev(T, s["dev"]), to_dev(p, s["dev"]), to_dev(Y, s["dev"]))
    torch.cuda.synchronize()
    try:
        for N, seed in ((2500, 74), (300, 75)):
            a, b = _both(s, N, seed)
            _same(a, b, f"FP8 {N} cells")
    finally:
        s["m"].set_precision(0)


def test_noalloc_rejects_batch_beyond_capacity(setup):
    import torch
    P = setup["P"]
    N = 1 << 15
    T, p, Y = chemgen.make_states(setup["mech"], "ch4", N=N, seed=76)
    dev = setup["dev"]
    Td, pd, Yd = to_dev(T, dev), to_dev(p, dev), to_dev(Y, dev)
    Y_before = Yd.clone()
    with pytest.raises(P.ChemError) as ei:
        setup["m"].step(setup["gm"], 1e-5, Td, pd, Yd, noalloc=True)
    torch.cuda.synchronize()
    assert "exceed" in str(ei.value)
    assert torch.equal(Yd, Y_before)  # nothing was launched
