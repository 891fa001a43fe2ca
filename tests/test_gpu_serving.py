"""GPU tests of the apply stage and of the serving loop, through the C ABI.

- the split-K apply (narrow right-hand sides) against the oracle's operator and against the
  MFMA GEMM apply, and its batch invariance (a column's result does not depend on the other
  columns of the launch: bitwise);
- the server: each request's Y against the oracle, bitwise equality of a request served alone
  and served inside a mix, admission by HBM footprint (refusal, queued build released by a
  removal), builds interleaved with applies, open-loop replay statistics.
"""
import time

import numpy as np
import pytest

import workloads as W
from oracle import nd_dtn, dst_dtn
from parity import assert_close

pytestmark = pytest.mark.gpu

# (n, leaf, kind): well-conditioned operators of several ring sizes (nb = 4(n - 1))
SMALL_OPS = [(40, 8, "laplace"), (64, 16, "cd"), (96, 16, "helm"), (130, 32, "cd")]


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def coeffs(n, kind, seed):
    rng = np.random.default_rng(seed)
    if kind == "laplace":
        return None, None, None
    if kind == "cd":
        return rng.uniform(-8, 8, n * n), rng.uniform(-8, 8, n * n), rng.uniform(0, 16, n * n)
    if kind == "helm":
        return None, None, np.full(n * n, -150.0)
    raise ValueError(kind)


@pytest.fixture(scope="module")
def small_ops(dtn):
    out = []
    for q, (n, leaf, kind) in enumerate(SMALL_OPS):
        b, c, d = coeffs(n, kind, 900 + q)
        op = dtn.build(n, b, c, d, leaf=leaf)
        out.append((op, nd_dtn(n, b, c, d, leaf=leaf)))
    yield out
    for op, _ in out:
        op.free()


def test_splitk_apply_vs_oracle_and_batch_invariance(dtn, small_ops):
    rng = np.random.default_rng(11)
    for op, Tref in small_ops:
        G = rng.uniform(-1, 1, (op.nb, 70))
        Y64 = op.apply(G[:, :64])
        assert_close(Y64, Tref @ G[:, :64], 1e-11, label=f"split-K nb={op.nb}")
        for k in (1, 2, 5, 16, 33):
            Yk = op.apply(G[:, :k])
            assert np.array_equal(Yk, Y64[:, :k]), f"nb={op.nb} k={k}: split-K result depends on the batch"
        # a column placed elsewhere in the batch gives the same bits
        Yr = op.apply(G[:, 7:40])
        assert np.array_equal(Yr, Y64[:, 7:40])
        # k = 70 runs the MFMA GEMM: same values to rounding
        Y70 = op.apply(G)
        assert_close(Y70[:, :64], Y64, 1e-14, label=f"GEMM vs split-K nb={op.nb}")


def test_splitk_apply_device_strided(dtn, small_ops):
    import torch
    op, Tref = small_ops[3]
    rng = np.random.default_rng(12)
    nb, k, ld = op.nb, 9, op.nb + 13
    Gh = rng.uniform(-1, 1, (nb, k))
    Gbig = torch.zeros((k, ld), dtype=torch.float64, device="cuda").t()
    Gbig[:nb] = torch.from_numpy(Gh).cuda()
    Ybig = torch.full((k, ld), 7.0, dtype=torch.float64, device="cuda").t()
    op.apply_device(Gbig[:nb], Ybig[:nb])
    torch.cuda.synchronize()
    Y = Ybig.cpu().numpy()
    assert_close(Y[:nb], Tref @ Gh, 1e-11, label="split-K strided")
    assert np.all(Y[nb:] == 7.0)      # padding rows untouched


def test_splitk_apply_full_size(dtn):
    """n = 1024 Helmholtz (20 wavelengths), the benchmark operator: narrow applies against the
    closed-form operator (conditioning-limited tolerance) and against the GEMM apply."""
    P = W.config("cfg3")
    op = dtn.build(P.n, P.b, P.c, P.d, leaf=P.leaf)
    try:
        Tref = dst_dtn(P.n, float(P.d[0]))
        G = P.G()[:, :80]
        Y1 = op.apply(G[:, :1])
        Y64 = op.apply(G[:, :64])
        Y80 = op.apply(G)
        assert np.array_equal(Y1, Y64[:, :1])
        assert_close(Y64, Tref @ G[:, :64], 1e-10, label="cfg3 split-K vs closed form")
        assert_close(Y80[:, :64], Y64, 1e-13, label="cfg3 GEMM vs split-K")
    finally:
        op.free()


def test_server_alone_vs_mix_bitwise(dtn, small_ops):
    rng = np.random.default_rng(21)
    srv = dtn.Server(budget_bytes=8 << 30, max_batch_cols=64)
    try:
        ids = [srv.add_op(op) for op, _ in small_ops]
        reqs = []
        for q in range(40):
            o = int(rng.integers(0, len(ids)))
            k = int(rng.integers(1, 33))
            reqs.append((o, rng.uniform(-1, 1, (small_ops[o][0].nb, k))))
        alone = []
        for o, G in reqs:
            Y, res = srv.wait(srv.submit_apply(ids[o], G))
            assert res["batch_cols"] == G.shape[1]
            alone.append(Y)
        tickets = [srv.submit_apply(ids[o], G) for o, G in reqs]
        batched = 0
        for (o, G), t, Ya in zip(reqs, tickets, alone):
            Y, res = srv.wait(t)
            batched += res["batch_cols"] > res["k"]
            assert np.array_equal(Y, Ya), "result in the mix differs from the result alone"
            assert_close(Y, small_ops[o][1] @ G, 1e-11, label="served in the mix")
        assert batched > 0, "no request was batched with another"
        st = srv.stats()
        assert st["applies_done"] == 80 and st["solves_done"] == 2 * sum(G.shape[1] for _, G in reqs)
    finally:
        srv.close()


def _wide_batches(srv, op_id, nb, ks, rng):
    """Submit requests of ks columns together (the slots fill up, so later ones batch), then each
    alone; returns (list of (G, Y batched, Y alone), number of requests that ran inside a batch wider
    than one 64-column group together with other requests)."""
    Gs = [rng.uniform(-1, 1, (nb, k)) for k in ks]
    tickets = [srv.submit_apply(op_id, G) for G in Gs]
    out, wide_mixed = [], 0
    for G, t in zip(Gs, tickets):
        Y, res = srv.wait(t)
        wide_mixed += res["batch_cols"] > max(64, res["k"])
        Ya, res_a = srv.wait(srv.submit_apply(op_id, G))
        assert res_a["batch_cols"] == G.shape[1]
        out.append((G, Y, Ya))
    return out, wide_mixed


def test_server_wide_batches_bitwise(dtn, small_ops):
    """Batches of up to 256 columns run as one split-K launch (up to four column groups per T tile):
    each request's Y is bitwise its result alone and matches the oracle; the ring sizes cover one
    split, several splits and a padded grid."""
    rng = np.random.default_rng(61)
    srv = dtn.Server(budget_bytes=8 << 30, max_batch_cols=256)
    try:
        for op, Tref in small_ops:
            out, wide_mixed = _wide_batches(srv, srv.add_op(op), op.nb, (50, 70, 3, 90, 43, 17, 64, 1) * 4, rng)
            assert wide_mixed > 0, "no request was served inside a wide batch"
            for G, Y, Ya in out:
                assert np.array_equal(Y, Ya), f"nb={op.nb}: batched result differs from the result alone"
                assert_close(Y, Tref @ G, 1e-11, label=f"wide batch nb={op.nb}")
    finally:
        srv.close()


def test_server_wide_batches_full_ring(dtn):
    """The same at nb = 4096 (16 splits): Laplace n = 1025 against the closed form."""
    n = 1025
    op = dtn.build(n, leaf=32)
    srv = dtn.Server(budget_bytes=16 << 30, max_batch_cols=256)
    try:
        out, wide_mixed = _wide_batches(srv, srv.add_op(op), op.nb, (64, 100, 92, 30, 7, 128) * 3,
                                        np.random.default_rng(62))
        assert wide_mixed > 0, "no request was served inside a wide batch"
        Tref = np.asarray(dst_dtn(n, 0.0), dtype=np.float64)
        for G, Y, Ya in out:
            assert np.array_equal(Y, Ya)
            assert_close(Y, Tref @ G, 1e-10, label="wide batch nb=4096 vs closed form")
    finally:
        srv.close()
        op.free()


def test_server_admission_by_footprint(dtn):
    n, leaf = 40, 8
    nb = 4 * (n - 1)
    A = dtn.build(n, leaf=leaf)
    big = dtn.build(130, leaf=32)
    try:
        # measure the charge of one server-built operator (operator + plan workspace + staging)
        s1 = dtn.Server(budget_bytes=1 << 30, max_batch_cols=16)
        try:
            _, res = s1.wait(s1.submit_build(n, leaf=leaf))
            assert res["status"] == 0
            charge_build = s1.stats()["resident_bytes"]
        finally:
            s1.close()
        t_bytes = nb * nb * 8
        budget = charge_build + t_bytes // 2
        s2 = dtn.Server(budget_bytes=budget, max_batch_cols=16)
        try:
            a_id = s2.add_op(A)
            with pytest.raises(dtn.DtnError) as e:
                s2.add_op(big)                      # does not fit next to A
            assert e.value.code == dtn.DTN_EBUSY
            with pytest.raises(dtn.DtnError) as e:
                s2.submit_build(1024, leaf=32)      # can never fit
            assert e.value.code == dtn.DTN_EBUSY
            t = s2.submit_build(n, leaf=leaf)       # fits only once A is gone: queued
            time.sleep(0.5)
            assert not s2.poll(t)
            G = np.random.default_rng(3).uniform(-1, 1, (nb, 3))
            Ya, _ = s2.wait(s2.submit_apply(a_id, G))
            s2.remove_op(a_id)
            _, res = s2.wait(t)
            assert res["status"] == 0
            Yb, _ = s2.wait(s2.submit_apply(res["op_id"], G))
            assert np.array_equal(Ya, Yb)           # same problem, same kernels, same bits
            with pytest.raises(dtn.DtnError):
                s2.submit_apply(a_id, G)            # removed
            with pytest.raises(dtn.DtnError):
                s2.submit_apply(res["op_id"], np.zeros((nb, 17)))   # k > max_batch_cols
            assert s2.stats()["refused"] >= 2
        finally:
            s2.close()
    finally:
        A.free()
        big.free()


def test_server_builds_interleaved_with_applies(dtn, small_ops):
    rng = np.random.default_rng(31)
    n, leaf = 72, 8
    b, c, d = coeffs(n, "cd", 77)
    Tref = nd_dtn(n, b, c, d, leaf=leaf)
    srv = dtn.Server(budget_bytes=8 << 30, max_batch_cols=64)
    try:
        ids = [srv.add_op(op) for op, _ in small_ops]
        tb = srv.submit_build(n, b, c, d, leaf=leaf)
        work = []
        for q in range(30):
            o = q % len(ids)
            G = rng.uniform(-1, 1, (small_ops[o][0].nb, 1 + q % 7))
            work.append((o, G, srv.submit_apply(ids[o], G)))
        _, res = srv.wait(tb)
        assert res["status"] == 0
        new_id = res["op_id"]
        G = rng.uniform(-1, 1, (4 * (n - 1), 5))
        Y, _ = srv.wait(srv.submit_apply(new_id, G))
        assert_close(Y, Tref @ G, 1e-11, label="server-built operator")
        for o, Gq, t in work:
            Yq, _ = srv.wait(t)
            assert_close(Yq, small_ops[o][1] @ Gq, 1e-11, label="apply beside a build")
        assert srv.stats()["builds_done"] == 1
    finally:
        srv.close()


def test_server_replay_open_loop(dtn, small_ops):
    rng = np.random.default_rng(41)
    srv = dtn.Server(budget_bytes=8 << 30, max_batch_cols=64)
    try:
        ids = [srv.add_op(op) for op, _ in small_ops]
        sched, t = [], 0.0
        for q in range(300):
            t += rng.exponential(1.0 / 5000.0)
            o = int(rng.integers(0, len(ids)))
            sched.append((t, ids[o], rng.uniform(-1, 1, (small_ops[o][0].nb, int(rng.integers(1, 65))))))
        srv.reset_stats()
        tickets = srv.replay(sched)
        for (tq, o, G), tk in zip(sched, tickets):
            Y, res = srv.wait(tk)
            assert res["t_done_ns"] >= res["t_start_ns"] >= res["t_arrival_ns"] - 1_000_000
            assert_close(Y, small_ops[ids.index(o)][1] @ G, 1e-11, label="replayed request")
        st = srv.stats()
        assert st["applies_done"] == 300
        assert st["solves_done"] == sum(G.shape[1] for _, _, G in sched)
        assert 0 < st["p50_ms"] <= st["p99_ms"]
        assert st["solves_per_s"] > 0 and st["mean_batch_cols"] >= 1
    finally:
        srv.close()


def test_server_replay_with_build_requests(dtn, small_ops):
    """Build requests inside a replayed open-loop schedule: admitted by footprint, built beside the
    applies, resident when done (their operator matches the oracle), build latency reported."""
    rng = np.random.default_rng(51)
    n, leaf = 65, 16
    b, c, d = coeffs(n, "cd", 52)
    srv = dtn.Server(budget_bytes=8 << 30, max_batch_cols=64)
    try:
        ids = [srv.add_op(op) for op, _ in small_ops]
        sched, t = [], 0.0
        for q in range(120):
            t += rng.exponential(1.0 / 4000.0)
            if q in (30, 80):
                sched.append((t, "build", dict(n=n, b=b, c=c, d=d, leaf=leaf)))
                continue
            o = int(rng.integers(0, len(ids)))
            sched.append((t, ids[o], rng.uniform(-1, 1, (small_ops[o][0].nb, int(rng.integers(1, 33))))))
        srv.reset_stats()
        tickets = srv.replay(sched)
        built = []
        for item, tk in zip(sched, tickets):
            Y, res = srv.wait(tk)
            if item[1] == "build":
                assert res["status"] == 0 and res["op_id"] >= 0
                built.append(res["op_id"])
            else:
                assert_close(Y, small_ops[ids.index(item[1])][1] @ item[2], 1e-11, label="replayed apply")
        st = srv.stats()
        assert st["builds_done"] == 2 and st["build_p50_ms"] > 0 and st["build_p99_ms"] >= st["build_p50_ms"]
        assert st["applies_done"] == 118
        Tref = nd_dtn(n, b, c, d, leaf=leaf)
        G = rng.uniform(-1, 1, (4 * (n - 1), 3))
        for op_id in built:
            Y, _ = srv.wait(srv.submit_apply(op_id, G))
            assert_close(Y, Tref @ G, 1e-11, label="operator built by a replayed request")
            srv.remove_op(op_id)
    finally:
        srv.close()


def test_server_hbs_only_operator(dtn):
    """An operator kept as HBS factors only (dense T released) is served through the telescoping
    apply, charged at its factors' size."""
    n, leaf = 200, 16
    rng = np.random.default_rng(61)
    b, c, d = coeffs(n, "cd", 62)
    op = dtn.build(n, b, c, d, leaf=leaf)
    T = op.dense()
    # the same server holding the dense operator: identical staging, the dense T charged
    srv = dtn.Server(budget_bytes=1 << 30, max_batch_cols=64)
    try:
        oid = srv.add_op(op)
        dense_bytes = srv.stats()["resident_bytes"]
        srv.remove_op(oid)
    finally:
        srv.close()
    op.hbs_compress(1e-10, 64, drop_dense=True)
    srv = dtn.Server(budget_bytes=1 << 30, max_batch_cols=64)
    try:
        oid = srv.add_op(op)
        hbs_bytes = srv.stats()["resident_bytes"]
        print(f"resident bytes: dense {dense_bytes}, HBS only {hbs_bytes} (factors {op.hbs_info()['bytes']})")
        assert hbs_bytes < dense_bytes
        tickets = []
        for q in range(12):
            G = rng.uniform(-1, 1, (op.nb, 1 + q % 9))
            tickets.append((G, srv.submit_apply(oid, G)))
        for G, tk in tickets:
            Y, _ = srv.wait(tk)
            assert_close(Y, T @ G, 1e-9, label="HBS-only operator served")
        srv.remove_op(oid)
    finally:
        srv.close()
        op.free()
