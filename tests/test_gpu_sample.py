"""Parity of the GPU training-set sampler (chem_sample_states) with the
oracle of Sec. 3.1 on the same seeds and random numbers: the keep decisions
bit for bit (apart from samples whose ratios lie within rounding of a Table 1
limit), the states within a few ulps (the GPU's pow and fused multiply-adds
round differently from NumPy's)."""
import sys

import numpy as np
import pytest

import chemgen
from oracle import hfrd
from gpu_util import need_gpu, to_dev

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    return need_gpu()


@pytest.fixture(scope="module")
def mech():
    return chemgen.make_mechanism("ch4")


def _near_limit(mech, T, Y, rel=1e-12):
    """Samples whose temperature or element ratios sit within rounding of a
    limit: either side may be right."""
    hc, on, phi = hfrd.ratios(mech, Y)
    near = np.abs(T - hfrd.T_KEEP) <= rel * hfrd.T_KEEP
    for v, lims in ((hc, hfrd.HC), (on, hfrd.ON), (phi, hfrd.PHI)):
        for lim in lims:
            near |= np.abs(v - lim) <= rel * lim
    return near


def _run(dev, mech, P, T, p, Y, c, s, eq, air):
    ends = [None, None]
    if s is not None:
        ends = [to_dev(np.concatenate([[e[0], e[1]], e[2]]), dev) for e in (eq, air)]
    out = P.sample_states(P.Mechanism(mech), mech, to_dev(T, dev), to_dev(p, dev), to_dev(Y, dev),
                          to_dev(c, dev), None if s is None else to_dev(s, dev), *ends)
    import torch
    torch.cuda.synchronize()
    return [t.cpu().numpy() for t in out]


@pytest.mark.parametrize("N,mixfrac", [(4097, 0.1), (1, 0.0), (300, 1.0), (20000, 0.3)])
def test_sampler_parity(dev, mech, N, mixfrac):
    import paper_2312_05800_amd as P
    _say(f"[sampler] N={N} mixing share {mixfrac}")
    n2 = mech.index("N2")
    T, p, Y = chemgen.make_states(mech, "ch4", N=N, seed=808)
    c, s = chemgen.hfrd_randoms(mech.K, N, seed=809, mix_fraction=mixfrac)
    eq = chemgen.burnt_state(mech, 0.45, 1500.0)
    air = chemgen.air_state(mech)
    s_arg = s if mixfrac > 0 else None
    To, po, Yo, keep = _run(dev, mech, P, T, p, Y, c, s_arg, eq, air)
    Tr, pr, Yr, kr = hfrd.sample(mech, T, p, Y, c, s if s_arg is not None else np.full(N, -1.0),
                                 eq, air, n2)
    np.testing.assert_allclose(To, Tr, rtol=4e-16 * 4, atol=0)
    np.testing.assert_allclose(po, pr, rtol=4e-16 * 4, atol=0)
    # a few ulps of each y'^... plus the rescaling's sum
    np.testing.assert_allclose(Yo, Yr, rtol=2e-14, atol=1e-300)
    near = _near_limit(mech, Tr, Yr)
    agree = (keep.astype(bool) == kr) | near
    _say(f"  kept gpu {int(keep.sum())} oracle {int(kr.sum())} of {N}; near a limit {int(near.sum())}")
    assert agree.all()


def test_sampler_single_seed_has_zero_ranges(dev, mech):
    """With one seed the ranges are zero: T and p stay, y_N2 stays, the other
    species take their powers and the rescaling."""
    import paper_2312_05800_amd as P
    T, p, Y = chemgen.make_states(mech, "ch4", N=1, seed=9)
    c, _ = chemgen.hfrd_randoms(mech.K, 1, seed=10, mix_fraction=0.0)
    To, po, Yo, _ = _run(dev, mech, P, T, p, Y, c, None, None, None)
    assert To[0] == T[0] and po[0] == p[0]
    assert Yo[mech.index("N2"), 0] == Y[mech.index("N2"), 0]
    assert abs(Yo[:, 0].sum() - 1.0) <= 4e-16 * mech.K


def test_sampler_rejects_bad_arguments(dev, mech):
    import torch
    import paper_2312_05800_amd as P
    T, p, Y = chemgen.make_states(mech, "ch4", N=8, seed=9)
    c, s = chemgen.hfrd_randoms(mech.K, 8, seed=10, mix_fraction=0.5)
    gm = P.Mechanism(mech)
    # a mixing fraction without the end states is refused on the host
    with pytest.raises(P.ChemError):
        P.sample_states(gm, mech, to_dev(T, dev), to_dev(p, dev), to_dev(Y, dev), to_dev(c, dev),
                        to_dev(s, dev))
    torch.cuda.synchronize()
