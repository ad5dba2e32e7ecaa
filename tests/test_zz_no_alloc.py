"""mfs_p2p_stokes_noalloc (no device allocation inside the library: its
scratch is a fixed per-GPU array) against mfs_p2p_stokes, through the C ABI.

The two share the kernels, the work items and the launch shape, so their
outputs must agree bit for bit; each is also checked against the oracle's
FP64 pair loops at the pair-sum bars of tests/test_gpu_p2p.py (FP64 1e-12,
mixed 4 x the error of the float32 model of the same sum).  Two calls in a row, the second with a smaller input (the
scratch keeps the first call's contents), in both precisions, with and
without same-body pairs, ragged target blocks (301 targets per body), two
systems, and a request beyond the scratch that is refused before any launch.
"""
import ctypes

import numpy as np
import pytest
import torch

import mfs_workloads as W
from oracle import mfs_oracle as O
from oracle import fp32_model as M
from tests._helpers import rel_inf, structure

pytestmark = pytest.mark.gpu


def _mfs():
    from paper_2409_04215_amd import mfs
    return mfs


def _dev(x):
    return torch.tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


def _case(n_body, n_src, n_trg, seed, shift=0.0):
    wl = W.small_cluster(n_body, W.STOKES, n_src, n_trg, seed=seed)
    wl.centre = wl.centre + shift
    sp, tp, pp = structure(wl)
    X, tb = wl.world_points("trg")
    Y, sb = wl.world_points("src")
    f = np.random.default_rng(seed).standard_normal((Y.shape[0], 3))
    return sp, tp, pp, X, tb, Y, sb, f


def _joined(a, b):
    """Two independent systems in one call."""
    sp = np.array([0, len(a[1]) - 1, len(a[1]) - 1 + len(b[1]) - 1], np.int64)
    tp = np.concatenate([a[1], a[1][-1] + b[1][1:]])
    pp = np.concatenate([a[2], a[2][-1] + b[2][1:]])
    nb_a = len(a[1]) - 1
    return (sp, tp, pp, np.concatenate([a[3], b[3]]), np.concatenate([a[4], b[4] + nb_a]),
            np.concatenate([a[5], b[5]]), np.concatenate([a[6], b[6] + nb_a]), np.concatenate([a[7], b[7]]))


@pytest.mark.parametrize("prec_name", ["FP64", "MIXED"])
@pytest.mark.parametrize("skip", [True, False])
def test_noalloc_matches_stokes_twice(prec_name, skip):
    mfs = _mfs()
    prec = getattr(mfs, prec_name)
    flags = mfs.SKIP_SAME_BODY if skip else 0
    big = _joined(_case(5, 45, 301, seed=41), _case(3, 37, 70, seed=42, shift=100.0))
    small = _case(2, 20, 65, seed=43)
    for sp, tp, pp, X, tb, Y, sb, f in (big, small):
        x, y, fd = _dev(X), _dev(Y), _dev(f)
        ref_gpu = mfs.p2p_stokes(sp, tp, pp, x, y, fd, 1.0, flags, prec).cpu().numpy()
        got = mfs.p2p_stokes_noalloc(sp, tp, pp, x, y, fd, 1.0, flags, prec).cpu().numpy()
        # the oracle sums within each system only
        ref = np.zeros_like(ref_gpu)
        model = np.zeros_like(ref_gpu)
        first = M.ref_first_source(len(tp) - 1, sb, Y, tb, X)
        for s in range(len(sp) - 1):
            b0, b1 = sp[s], sp[s + 1]
            rt = slice(tp[b0], tp[b1])
            rs = slice(pp[b0], pp[b1])
            ref[rt] = O.p2p(O.STOKES, X[rt], tb[rt], Y[rs], sb[rs], f[rs], 1.0, skip)
            model[rt] = M.pair_sum(O.STOKES, X[rt], tb[rt], Y[rs], sb[rs], f[rs], first, skip)
        bar = 1e-12 if prec == mfs.FP64 else M.bar(rel_inf(model, ref))
        e = rel_inf(got, ref)
        print(f"{prec_name} skip={skip} targets={X.shape[0]} noalloc vs p2p_stokes max diff "
              f"{np.abs(got - ref_gpu).max():.1e}, vs oracle {e:.2e}")
        assert np.array_equal(got, ref_gpu)
        assert e <= bar


def test_noalloc_accumulate_and_limits():
    mfs = _mfs()
    sp, tp, pp, X, tb, Y, sb, f = _case(4, 30, 100, seed=44)
    x, y, fd = _dev(X), _dev(Y), _dev(f)
    base = torch.full((X.shape[0], 3), 0.25, dtype=torch.float64, device="cuda")
    out = base.clone()
    mfs.p2p_stokes_noalloc(sp, tp, pp, x, y, fd, 1.0, mfs.SKIP_SAME_BODY | mfs.ACCUMULATE, mfs.MIXED, out=out)
    plain = mfs.p2p_stokes_noalloc(sp, tp, pp, x, y, fd, 1.0, mfs.SKIP_SAME_BODY, mfs.MIXED)
    assert torch.equal(out, base + plain)
    # 2.2e6 targets in one body need more work items (and scratch) than the entry
    # point holds: refused on the host, the output untouched
    n_t = 2_200_000
    tp2 = np.array([0, n_t], np.int64)
    pp2 = np.array([0, 1], np.int64)
    sp2 = np.array([0, 1], np.int64)
    xs = torch.zeros((n_t, 3), dtype=torch.float64, device="cuda")
    ys = torch.ones((1, 3), dtype=torch.float64, device="cuda")
    fs = torch.ones((1, 3), dtype=torch.float64, device="cuda")
    o = torch.full((n_t, 3), 7.0, dtype=torch.float64, device="cuda")
    with pytest.raises(mfs.MfsError) as err:
        mfs.p2p_stokes_noalloc(sp2, tp2, pp2, xs, ys, fs, 1.0, 0, mfs.MIXED, out=o)
    assert err.value.status == mfs.MFS_EINVAL
    assert bool((o == 7.0).all())
