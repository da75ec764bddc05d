"""GPU helix fit (trk_fit) against the FP64 oracle on the same labels: the
generator's particles as candidates (tiny and pile-up-200 events) and the
chain's own labels; capacity and label errors."""
import numpy as np
import pytest
import torch

from gen import TINY, MU200, make_weights, generate_event
from oracle import fit as OF

pytestmark = pytest.mark.gpu


def _truth_labels(ev):
    lab = np.arange(ev.n)
    order = np.argsort(ev.pid, kind="stable")
    pid = ev.pid[order]
    starts = np.flatnonzero(np.r_[True, pid[1:] != pid[:-1]])
    for a, b in zip(starts, np.r_[starts[1:], len(pid)]):
        if pid[a] > 0:
            idx = order[a:b]
            lab[idx] = idx.min()
    return lab


def _compare(par, ref):
    assert par.shape == ref.shape
    ok = ~np.isnan(ref[:, 0])
    assert np.array_equal(np.isnan(par[:, 0]), ~ok)
    p, r = par[ok], ref[ok]
    assert np.max(np.abs(p[:, 0] / r[:, 0] - 1.0)) < 1e-6          # pT
    dphi = (p[:, 1] - r[:, 1] + np.pi) % (2 * np.pi) - np.pi
    assert np.max(np.abs(dphi)) < 1e-7
    assert np.max(np.abs(p[:, 2] - r[:, 2])) < 1e-6                # eta
    assert np.max(np.abs(p[:, 3] - r[:, 3])) < 1e-5                # z0, mm
    assert np.array_equal(p[:, 4], r[:, 4])                        # charge
    assert np.max(np.abs(p[:, 5] - r[:, 5]) / np.maximum(1.0, np.abs(r[:, 5]))) < 1e-6


@pytest.fixture(scope="module")
def pipe():
    from paper_2501_05520_amd.trk import Pipeline
    p = Pipeline(MU200, make_weights(MU200, 0), "fp32", max_hits=110000 + 64)
    yield p
    p.close()


@pytest.mark.parametrize("mu", [1, 200])
def test_fit_truth_candidates(pipe, mu):
    from paper_2501_05520_amd import trk
    ev = generate_event(40 + mu, mu)
    lab = _truth_labels(ev)
    x = torch.as_tensor(ev.x, device="cuda")
    l = torch.as_tensor(lab.astype(np.int32), device="cuda")
    cl, cn, par = trk.trk_fit(pipe.ctx, x, l, min_hits=3, b_field=2.0)
    rl, rn, rp = OF.fit_candidates(ev.x, lab, min_hits=3, b_field=2.0)
    assert np.array_equal(cl.cpu().numpy(), rl) and np.array_equal(cn.cpu().numpy(), rn)
    _compare(par.cpu().numpy(), rp)
    # and the generated particles come back
    pid = ev.pid[rl] - 1
    assert np.max(np.abs(par.cpu().numpy()[:, 0] / ev.truth["pt"][pid] - 1.0)) < 1e-3


def test_fit_chain_labels():
    from paper_2501_05520_amd.trk import Pipeline
    from paper_2501_05520_amd import trk
    nets = make_weights(TINY, 0)
    p = Pipeline(TINY, nets, "fp32", max_hits=8192)
    ev = generate_event(5, 2)
    labels, _ = p.event(ev.x)
    x = torch.as_tensor(ev.x, device="cuda")
    cl, cn, par = trk.trk_fit(p.ctx, x, labels, min_hits=3)
    rl, rn, rp = OF.fit_candidates(ev.x, labels.cpu().numpy(), min_hits=3)
    assert np.array_equal(cl.cpu().numpy(), rl) and np.array_equal(cn.cpu().numpy(), rn)
    _compare(par.cpu().numpy(), rp)
    # capacity and bad labels are reported, not truncated or read
    lab2 = torch.as_tensor(_truth_labels(ev).astype(np.int32), device="cuda")   # 100 candidates
    with pytest.raises(trk.TrkError) as e:
        trk.trk_fit(p.ctx, x, lab2, min_hits=3, cap=10)
    assert e.value.status == -3
    bad = labels.clone()
    bad[0] = ev.n + 5
    with pytest.raises(trk.TrkError) as e:
        trk.trk_fit(p.ctx, x, bad, min_hits=3)
    assert e.value.status == -1
    p.close()
