"""Served nonlinear heat solves (wq_server_*): continuous admission on concurrent slots.

* A request's result is the same alone and in a mix with other requests running on the
  device at the same time (the kernels sum in fixed orders: identical bits).
* A served result agrees with the oracle's Newton solve of the same problem (the oracle
  computes its own weights and solves directly: agreement to the solver tolerance over
  the weights' conditioning).
* Admission follows the HBM budget: with room for one request at a time they run one
  after the other; a request larger than the whole budget is refused.
* A domain's setup (mesh, points, weights) is held after its request: a later request on
  the same domain takes it over with bit-identical results, and an idle setup is released
  when a request needs its room.
"""
import numpy as np
import pytest

import fixtures as fx
import oracle as O
from oracle import heat as H

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _wq():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2605_29334_amd.wq as W
    return W


@pytest.fixture(scope="module")
def pool():
    print("[gpu] server pool", flush=True)
    return [fx.fixture_grid(8, displace=0.05, seed=11), fx.fixture_half_strip(),
            fx.fixture_eps(32, 0.02, (3, 5, 6), seed=5), fx.fixture_grid(12, displace=0.05, seed=3)]


# conductivities bounded away from zero on the solution's range (T* in [0, 1)); k = sin(pi T)
# vanishes at the initial state T = 0 and is exercised by the tangent parity tests instead
KINDS = [(H.K_QUADRATIC, 1.0, 1.0), (H.K_EXP, 1.0, -1.0), (H.K_LINEAR, 1.0, 0.0), (H.K_LINEAR, 1.0, 0.5)]


def _requests(pool):
    return [(pool[i % len(pool)], KINDS[i % len(KINDS)], 0.25 + 0.05 * i) for i in range(6)]


def _submit(S, req):
    F, k, dt = req
    return S.submit(F, F["dir1"], dt, 2, k=k)


def test_same_result_alone_and_in_the_mix(pool):
    W = _wq()
    reqs = _requests(pool)
    S = W.Server(8 << 30, 3)
    alone = []
    for r in reqs:
        T, res = S.poll(_submit(S, r))
        assert res["status"] == 0 and res["residual"] <= 1e-10, res
        alone.append(T)
    tickets = [_submit(S, r) for r in reqs]
    mixed = [S.poll(t) for t in tickets]
    S.close()
    overlap = any(b[1]["started"] < a[1]["finished"] for a, b in zip(mixed, mixed[1:]))
    lat = np.array([m[1]["finished"] - m[1]["submitted"] for m in mixed])
    print(f"[gpu] mix of {len(reqs)}: overlapped={overlap}, latency p50 {np.percentile(lat, 50):.3f} s "
          f"p99 {np.percentile(lat, 99):.3f} s")
    assert overlap
    for a, (T, res) in zip(alone, mixed):
        assert res["status"] == 0
        assert np.array_equal(a, T)


def test_served_result_matches_oracle(pool):
    W = _wq()
    F = pool[0]
    kind, a, b = KINDS[0]
    S = W.Server(4 << 30, 2)
    T, res = S.poll(S.submit(F, F["dir1"], 0.5, 2, k=(kind, a, b), cg_rtol=1e-12))
    S.close()
    R = O.setup(F, families=("mass", "x", "y"))
    pat, data, Wo = R["pat"], R["data"], R["W"]
    n = F["n_fn"]
    x = H.points_x(data)
    k, _ = H.conductivity(kind, a, b)
    _, f = H.manufactured(kind, a, b)
    To, Tdo = np.zeros(n), np.zeros(n)
    for s in range(2):
        To, Tdo, it, _ = H.heat_step(F, pat, data, Wo, To, Tdo, 0.5, 1.0, k, f(x, 0.5 * (s + 1)),
                                     F["dir1"].astype(bool), np.zeros(n))
    rel = np.abs(T - To).max() / np.abs(To).max()
    print(f"[gpu] served vs oracle: rel diff {rel:.2e}, newton {res['newton_iters']}, cg {res['cg_iters']}")
    assert rel < 1e-8


def test_admission_respects_the_budget(pool):
    W = _wq()
    # three requests of the same mesh (equal estimates)
    reqs = [(pool[0], KINDS[i], 0.3 + 0.1 * i) for i in range(3)]
    probe = W.Server(8 << 30, 1)
    est = []
    for r in reqs:
        _, res = probe.poll(_submit(probe, r))
        est.append(res["hbm_estimate"])
    probe.close()
    # room for the largest request but not for two: they must run one at a time
    S = W.Server(int(max(est) * 1.5), 3)
    out = [S.poll(t) for t in [_submit(S, r) for r in reqs]]
    S.close()
    for (_, a), (_, b) in zip(out, out[1:]):
        assert b["started"] >= a["finished"] - 1e-6, (a, b)


def test_request_larger_than_budget_is_refused(pool):
    W = _wq()
    S = W.Server(1 << 20, 1)
    with pytest.raises(W.WQError) as e:
        _submit(S, _requests(pool)[0])
    S.close()
    assert e.value.status == -2


def test_held_setup_is_reused_with_identical_results(pool):
    W = _wq()
    req = (pool[3], KINDS[0], 0.3)
    S = W.Server(8 << 30, 1)
    T1, r1 = S.poll(_submit(S, req))
    T2, r2 = S.poll(_submit(S, req))
    S.close()
    print(f"[gpu] held setup: first {r1['finished'] - r1['started']:.3f} s, reused {r2['finished'] - r2['started']:.3f} s")
    assert r1["status"] == 0 and r2["status"] == 0
    assert r1["setup_reused"] == 0 and r2["setup_reused"] == 1
    assert np.array_equal(T1, T2)


def test_idle_setup_is_released_when_room_is_needed(pool):
    W = _wq()
    a, b = (pool[0], KINDS[0], 0.3), (pool[3], KINDS[0], 0.3)
    probe = W.Server(8 << 30, 1)
    ea = probe.poll(_submit(probe, a))[1]["hbm_estimate"]
    eb = probe.poll(_submit(probe, b))[1]["hbm_estimate"]
    probe.close()
    # room for one held setup at a time: b releases a's idle setup, a is then rebuilt
    S = W.Server(int(max(ea, eb) * 1.5), 1)
    Ta1, r1 = S.poll(_submit(S, a))
    _, r2 = S.poll(_submit(S, b))
    Ta2, r3 = S.poll(_submit(S, a))
    S.close()
    assert [r["status"] for r in (r1, r2, r3)] == [0, 0, 0]
    assert [r["setup_reused"] for r in (r1, r2, r3)] == [0, 0, 0]
    assert np.array_equal(Ta1, Ta2)


def test_requests_without_setup_reuse(pool):
    """reuse_setup = 0: the same domain is set up again from scratch (nothing held,
    nothing taken over) with bit-identical results; the exact tangent is served too and
    takes fewer Newton iterations than the symmetric one on the same request."""
    W = _wq()
    F = pool[3]
    S = W.Server(8 << 30, 1)
    T1, r1 = S.poll(S.submit(F, F["dir1"], 0.3, 2, k=KINDS[0], reuse_setup=False))
    T2, r2 = S.poll(S.submit(F, F["dir1"], 0.3, 2, k=KINDS[0], reuse_setup=False))
    T3, r3 = S.poll(S.submit(F, F["dir1"], 0.3, 2, k=KINDS[0], reuse_setup=False, tangent=W.TANGENT_EXACT))
    S.close()
    assert [r["status"] for r in (r1, r2, r3)] == [0, 0, 0]
    assert [r["setup_reused"] for r in (r1, r2, r3)] == [0, 0, 0]
    assert np.array_equal(T1, T2)
    print(f"[gpu] served Newton iterations: symmetric {r1['newton_iters']}, exact {r3['newton_iters']}")
    assert r3["newton_iters"] < r1["newton_iters"]
    assert np.abs(T3 - T1).max() <= 1e-8 * np.abs(T1).max()


def test_joined_requests_agree_with_alone(pool):
    """Joining (wq_server_set_join): requests queued together with the same parameters run
    as one union of their meshes. With one slot, the requests submitted while the first one
    runs are joined at the next admission; each reports the union's size, and, each mesh
    being solved as a segment of its own (its reductions in the order they take alone, its
    own Newton and Krylov stops), its temperature, iteration counts and residual are bit for
    bit those of the request run alone. A request with other heat parameters is not joined."""
    W = _wq()
    same = [(pool[i % len(pool)], KINDS[0], 0.25) for i in range(6)]
    odd = (pool[1], KINDS[1], 0.3)
    S = W.Server(8 << 30, 1)
    alone = [S.poll(_submit(S, r)) for r in same + [odd]]
    with pytest.raises(W.WQError):
        S.set_join(0)
    with pytest.raises(W.WQError):
        S.set_join(4, -1)
    S.close()
    S = W.Server(8 << 30, 1)
    S.set_join(8)
    tickets = [_submit(S, r) for r in same + [odd]]
    out = [S.poll(t) for t in tickets]
    S.close()
    joined = [res["joined"] for _, res in out]
    print(f"[gpu] joined sizes {joined}", flush=True)
    assert all(res["status"] == 0 for _, res in out)
    assert max(joined[:-1]) >= 2 and joined[-1] == 1
    for (Ta, ra), (Tj, rj) in zip(alone, out):
        assert rj["n_rows"] == ra["n_rows"] and rj["nnz"] == ra["nnz"]
        assert rj["residual"] <= 1e-10
        err = np.abs(Tj - Ta).max()
        print(f"[gpu] joined {rj['joined']}: max |T_joined - T_alone| {err:.2e} (max |T| {np.abs(Ta).max():.2f})")
        assert np.array_equal(Tj, Ta)
        assert (rj["newton_iters"], rj["cg_iters"], rj["residual"]) == (ra["newton_iters"], ra["cg_iters"],
                                                                         ra["residual"])
        if rj["joined"] > 1:  # (alone, it may take over a setup held by an earlier request)
            assert rj["setup_reused"] == 0


def test_join_row_cap_keeps_requests_apart(pool):
    """A union may not exceed max_rows: with a cap below any two meshes together, no
    request is joined and every result is bit-identical to the request run alone."""
    W = _wq()
    reqs = [(pool[i % len(pool)], KINDS[0], 0.25) for i in range(4)]
    S = W.Server(8 << 30, 1)
    alone = [S.poll(_submit(S, r))[0] for r in reqs]
    S.close()
    S = W.Server(8 << 30, 1)
    S.set_join(8, max_rows=min(F["n_fn"] for F in pool))
    out = [S.poll(t) for t in [_submit(S, r) for r in reqs]]
    S.close()
    assert [res["joined"] for _, res in out] == [1] * len(reqs)
    for Ta, (Tj, _) in zip(alone, out):
        assert np.array_equal(Tj, Ta)
