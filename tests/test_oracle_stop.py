"""Pins of the oracle's learned-stop path: the 16 state features and labels
against a hand trace, against the observable state of searches stopped at
each hop, and the stop rule against its limiting thresholds."""
import json
from pathlib import Path

import numpy as np
import pytest

import oracle
import synth

GOLD = Path(__file__).resolve().parent / "golden"
F32 = np.float32


def f32expr(s):
    """FP32 value of a fixture expression: a number, 'a/b' or 'sqrt(a)'."""
    s = s.strip()
    if s.startswith("sqrt(") and s.endswith(")"):
        return np.sqrt(F32(float(s[5:-1])))
    if "/" in s:
        a, b = s.split("/")
        return F32(float(a)) / F32(float(b))
    return F32(float(s))


def _run_toy(c, adj, **kw):
    pts = np.array(c["points"], np.float32).reshape(-1, 1)
    if "query_vertex" in c:
        return oracle.range_search_indexed(pts, adj, [c["query_vertex"]], c["k"], c["eps"], **kw)
    q = np.array([[c["query"]]], np.float32)
    return oracle.range_search(pts, adj, q, np.array([c["seeds"]]), c["k"], c["eps"], **kw)


def test_hand_traced_features_and_labels():
    g = json.loads((GOLD / "stop_features_toy.json").read_text())
    adj = np.array(g["adj"], np.int32)
    for c in g["cases"]:
        nrows = len(c["rows"])
        ids, ds, st, tr = _run_toy(c, adj, trace_rows=nrows + 2, trace_interval=1)
        assert st[0, 0] == c["hops"], c["trace"]
        for i, row in enumerate(c["rows"]):
            want = np.array([f32expr(v) for v in row], np.float32)
            got = tr[0, i, :16]
            assert (got == want).all(), (c["trace"], i, got.tolist(), want.tolist())
            assert tr[0, i, 16] == c["labels"][i], (c["trace"], i)
            assert tr[0, i, 18] == i + 1
        assert (tr[0, nrows:, 16] == -1).all()


def _random_model(seed, tau, interval, tau_long=None, long_hops=0):
    r = synth.rng(seed)
    p = (r.standard_normal(5313) * 0.3).astype(np.float32)
    return oracle.StopModel(oracle.bf16_encode(p), np.zeros(16, np.float32),
                            np.ones(16, np.float32), tau, interval, tau_long, long_hops)


_G = {}


def graph():
    if "g" not in _G:
        x = synth.small_int(3, 1500, 24, hi=64)
        adj, _, _ = oracle.build_graph(x, 16, k_ext=32, eps_ext=0.2, k_opt=16)
        _G["g"] = (x, adj)
    return _G["g"]


def test_tau_one_never_stops_and_tau_zero_stops_at_first_checkpoint():
    x, adj = graph()
    q = synth.small_int(4, 120, 24, hi=64)
    plain = oracle.range_search(x, adj, q, [0], 10, 0.1)
    never = oracle.range_search(x, adj, q, [0], 10, 0.1, stop=_random_model(1, 1.0, 4))
    assert (never[0] == plain[0]).all() and (never[2][:, :2] == plain[2][:, :2]).all()
    assert (never[2][:, 3] & 16 == 0).all()
    for itv in (1, 3, 8):
        now = oracle.range_search(x, adj, q, [0], 10, 0.1, stop=_random_model(1, 0.0, itv))
        long_enough = plain[2][:, 0] >= itv
        assert (now[2][long_enough, 0] == itv).all()
        assert (now[2][long_enough, 3] & 16 != 0).all()
        assert (now[0][~long_enough] == plain[0][~long_enough]).all()


def test_long_query_threshold_applies_from_its_hop():
    x, adj = graph()
    q = synth.small_int(5, 120, 24, hi=64)
    plain = oracle.range_search(x, adj, q, [0], 10, 0.1)
    m = _random_model(2, 1.0, 4, tau_long=0.0, long_hops=10)
    got = oracle.range_search(x, adj, q, [0], 10, 0.1, stop=m)
    first = 12  # the first checkpoint (multiple of 4) at or after hop 10
    reach = plain[2][:, 0] >= first
    assert reach.any() and (got[2][reach, 0] == first).all()
    assert (got[0][~reach] == plain[0][~reach]).all()


def _stopped_at(x, adj, q, k, eps, h, **kw):
    """The search of one query ended at the checkpoint of hop h (tau = 0)."""
    m = _random_model(9, 0.0, h)
    return oracle.range_search(x, adj, q[None], [0], k, eps, stop=m, **kw)


@pytest.mark.parametrize("k,eps", [(10, 0.0), (10, 0.1), (4, 0.2)])
def test_labels_agree_with_searches_stopped_at_each_row(k, eps):
    # label of the row at hop h = 1 exactly when the first min(k, 10) results of
    # the search stopped at hop h are already the final ones
    x, adj = graph()
    q = synth.small_int(6, 12, 24, hi=64)
    itv = 3
    ids, ds, st, tr = oracle.range_search(x, adj, q, [0], k, eps, trace_rows=64,
                                          trace_interval=itv)
    t = min(k, 10)
    checked = 0
    for i in range(q.shape[0]):
        for row in range(64):
            lab = tr[i, row, 16]
            if lab < 0:
                break
            h = itv * (row + 1)
            sid, sds, sst = _stopped_at(x, adj, q[i], k, eps, h)
            same = sid[0, :t].tolist() == ids[i, :t].tolist() and (sds[0, :t] == ds[i, :t]).all()
            assert lab == (1.0 if same else 0.0), (i, row)
            checked += 1
    assert checked > 40


def test_features_agree_with_the_state_of_stopped_searches():
    # features 0-6 and 14 from the outputs of the searches stopped at every hop:
    # evaluations, R (distances), r, and when R's front, first entry and r changed
    x, adj = graph()
    q = synth.small_int(7, 4, 24, hi=64)
    k, eps, itv = 6, 0.1, 2
    ids, ds, st, tr = oracle.range_search(x, adj, q, [0], k, eps, trace_rows=200,
                                          trace_interval=itv)
    for i in range(q.shape[0]):
        H = int(st[i, 0])
        states = {}
        for h in range(1, H + 1):
            sid, sds, sst = _stopped_at(x, adj, q[i], k, eps, h)
            states[h] = (sid[0], sds[0], int(sst[0, 1]))
        dseed = F32(oracle.dist32(x[0], q[i]))

        def r_of(h):
            sd = states[h][1]
            return sd[k - 1] if np.isfinite(sd[k - 1]) and (states[h][0] >= 0).sum() == k else F32(np.inf)

        def last_change(h, key):
            for j in range(h - 1, 0, -1):
                if key(j + 1) != key(j):
                    return j
            return 0

        front = lambda h: (tuple(states[h][0][:min(k, 10)]), tuple(states[h][1][:min(k, 10)]))
        first = lambda h: (states[h][0][0], states[h][1][0])
        for row in range(H // itv):
            h = itv * (row + 1)
            f = tr[i, row, :16]
            sid, sd, ev = states[h]
            d1, dk = sd[0], sd[k - 1] if sid[k - 1] >= 0 else sd[(sid >= 0).sum() - 1]
            assert f[0] == np.sqrt(F32(h)) and f[1] == np.sqrt(F32(ev))
            assert f[2] == (d1 / dk if dk > 0 else F32(1))
            assert f[3] == (d1 / dseed if dseed > 0 else F32(1))
            rp = r_of(h - itv) if h > itv else F32(np.inf)
            r = r_of(h)
            assert f[4] == (r / rp if np.isfinite(r) and np.isfinite(rp) and rp > 0 else F32(1))
            # a change during hop j shows in the state stopped at hop j + 1
            assert f[5] == np.sqrt(F32(h - last_change(h, front)))
            assert f[6] == np.sqrt(F32(h - last_change(h, first)))
            assert f[14] == np.sqrt(F32(h - last_change(h, r_of)))
            assert f[11] == F32(eps) and f[12] == np.sqrt(F32(k)) and f[13] == 0 and f[15] == 1
            assert 0 <= f[7] <= 1 and 0 <= f[8] <= f[7] + 1e-7 and 0 <= f[9] <= 1


def test_stop_happens_at_the_first_checkpoint_whose_logit_passes():
    # the trace rows of the plain search, standardised and fed to the BF16
    # network, predict the hop at which the stopped search ends
    x, adj = graph()
    q = synth.small_int(8, 80, 24, hi=64)
    k, eps, itv = 10, 0.1, 4
    ids, ds, st, tr = oracle.range_search(x, adj, q, [0], k, eps, trace_rows=128,
                                          trace_interval=itv)
    rows = tr[:, :, :16].reshape(-1, 16)
    mean = rows.mean(0).astype(np.float32)
    sd = rows.std(0).astype(np.float32)
    istd = np.where(sd > 1e-6, 1 / np.maximum(sd, 1e-6), 0).astype(np.float32)
    r = synth.rng(12)
    w = oracle.bf16_encode((r.standard_normal(5313) * 0.3).astype(np.float32))
    fs = ((tr[:, :, :16] - mean) * istd).astype(np.float32)
    z = oracle.mlp_logits_bf16(w, fs.reshape(-1, 16)).reshape(q.shape[0], 128)
    zt = np.float32(np.log(np.float32(0.6) / (np.float32(1) - np.float32(0.6))))
    m = oracle.StopModel(w, mean, istd, 0.6, itv)
    got = oracle.range_search(x, adj, q, [0], k, eps, stop=m)
    stopped = 0
    for i in range(q.shape[0]):
        valid = tr[i, :, 16] >= 0
        hit = np.nonzero(valid & (z[i] >= zt))[0]
        if len(hit):
            assert got[2][i, 0] == itv * (hit[0] + 1) and got[2][i, 3] & 16
            stopped += 1
        else:
            assert got[2][i, 0] == st[i, 0] and not got[2][i, 3] & 16
    assert 0 < stopped < q.shape[0]
