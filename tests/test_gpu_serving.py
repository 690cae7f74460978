"""Batched and served jobs (through the C ABI): each job's result inside a mix
is identical to its result alone, under both scheduling policies, with jobs
admitted by arena memory and submitted while others run."""
import time

import numpy as np
import pytest

import pps_workloads as W
from gpu_helpers import observed, require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    return require_gpu()


@pytest.fixture(scope="module")
def P(torch):
    import paper_1902_09046_amd as P
    return P


def mixed_jobs(P, n_jobs=14, seed=5):
    """ABC (closest 1 % and fixed eps) and p-value jobs of different N, step
    count, seed and lambda."""
    rng = np.random.default_rng(seed)
    ob = observed()["logistic_S1000"]
    lam = W.lambda_grid(64)
    jobs, meta = [], []
    for i in range(n_jobs):
        n = int(rng.integers(700, 30000))
        steps = int(rng.choice([200, 400, 1000, 2000]))
        first = int(rng.integers(0, 10**6))
        s = P.make_sampling(n, first, 100 + i)
        if i % 2 == 0:
            spec = W.logistic_spec(steps=steps)
            if i % 4 == 0:
                jobs.append(P.make_abc_job(spec, ob["y_obs"], s, P.PPS_EPS_TOP_FRACTION, 0.01))
                meta.append(("abc_top", spec, s, 0.01))
            else:
                jobs.append(P.make_abc_job(spec, ob["y_obs"], s, P.PPS_EPS_FIXED, 55.0, capacity=4000))
                meta.append(("abc_fixed", spec, s, 55.0))
        else:
            spec = W.pvalue_spec(steps=steps)
            l = float(lam[int(rng.integers(0, 64))])
            jobs.append(P.make_pvalue_job(spec, 0, P.PPS_LOGNORMAL, l, s, ob["t_obs"]))
            meta.append(("pvalue", spec, s, l))
    return jobs, meta


def alone(P, meta):
    """Each job run by itself through the synchronous entry points."""
    ob = observed()["logistic_S1000"]
    out = []
    for kind, spec, s, arg in meta:
        if kind.startswith("abc"):
            mode = P.PPS_EPS_TOP_FRACTION if kind == "abc_top" else P.PPS_EPS_FIXED
            r = P.abc(spec, ob["y_obs"], s.seed, s.first_draw, s.n_draws, mode, arg,
                      capacity=None if mode == P.PPS_EPS_TOP_FRACTION else 4000)
            out.append(r)
        else:
            c, _ = P.prior_pred_pvalue(spec, 0, P.PPS_LOGNORMAL, [arg], s, ob["t_obs"])
            out.append({"count_ge": int(c[0])})
    return out


def assert_same(P, res, ref, arena):
    assert res.status in (P.PPS_OK, P.PPS_ETRUNC)
    if "count_ge" in ref:
        assert res.count_ge == ref["count_ge"]
        return
    assert res.abc.n_accepted == ref["n_accepted"]
    assert res.abc.eps_used == ref["eps_used"]
    np.testing.assert_array_equal(np.array(res.abc.mean[:3]), ref["mean"][:3])
    np.testing.assert_array_equal(np.array(res.abc.var[:3]), ref["var"][:3])
    idx, th, d = P.records(res, arena, 3)
    np.testing.assert_array_equal(idx, ref["idx"].cpu().numpy().astype(np.uint64))
    np.testing.assert_array_equal(th, ref["theta"].cpu().numpy())
    np.testing.assert_array_equal(d, ref["dist"].cpu().numpy())


@pytest.fixture(scope="module")
def arena(torch):
    return torch.empty(256 << 20, dtype=torch.uint8, device="cuda")


@pytest.mark.parametrize("policy", ["batched", "plain"])
def test_batch_results_equal_alone(P, torch, arena, policy):
    jobs, meta = mixed_jobs(P)
    ref = alone(P, meta)
    pol = P.PPS_POLICY_BATCHED if policy == "batched" else P.PPS_POLICY_PLAIN
    cfg = P.make_server_config(arena, epoch_ms=0.5, policy=pol)
    res = P.pps_run_batch(jobs, cfg)
    for r, f in zip(res, ref):
        assert_same(P, r, f, arena)


def test_server_mix_equals_alone(P, torch, arena):
    jobs, meta = mixed_jobs(P, n_jobs=16, seed=9)
    ref = alone(P, meta)
    cfg = P.make_server_config(arena, epoch_ms=1.0, max_active=64)
    with P.Server(cfg) as srv:
        ids = []
        for j in jobs:
            ids.append(srv.submit(j))
            time.sleep(0.0005)  # later jobs arrive while earlier ones run
        deadline = time.time() + 60
        done = {}
        while len(done) < len(ids) and time.time() < deadline:
            for i, jid in enumerate(ids):
                if i in done:
                    continue
                rc, r = srv.poll(jid)
                if rc != P.PPS_PENDING:
                    done[i] = r
            time.sleep(0.001)
        assert len(done) == len(ids)
        for i in range(len(ids)):
            assert_same(P, done[i], ref[i], arena)
            assert done[i].t_submit <= done[i].t_admit <= done[i].t_done
        st = srv.stats()
        assert st.completed == len(ids) and st.submitted == len(ids)
        assert 0 < st.latency_p50_s <= st.latency_p99_s
        assert st.epochs >= 1
        for jid in ids:
            assert srv.release(jid) == P.PPS_OK
        assert srv.release(ids[0]) == P.PPS_ENOTFOUND
        with pytest.raises(P.PPSError):
            srv.poll(ids[0])


def every_model_jobs(P):
    """Closest-fraction and fixed-eps ABC jobs of the toggle-switch and
    tuberculosis models, with logistic ABC and p-value jobs between them:
    (job, (spec, y_obs, sampling, mode, eps_or_frac, capacity)) pairs."""
    g = observed()
    models = [
        (W.toggle_spec(n_cells=400, steps=100), g["toggle_C8000_T600"]["y_obs"], 300),
        (W.tb_spec(n_stop=300, n_sample=100, max_events=20000), g["tb_K10000_n473"]["y_obs"], 700),
    ]
    out = []
    for k, (spec, y, n) in enumerate(models):
        s = P.make_sampling(n, 1000 * k, 40 + k)
        out.append((P.make_abc_job(spec, y, s, P.PPS_EPS_TOP_FRACTION, 0.05),
                    (spec, y, s, P.PPS_EPS_TOP_FRACTION, 0.05, None)))
        # a tolerance that keeps about a third of the job's draws
        s2 = P.make_sampling(n // 2, 77, 50 + k)
        eps = P.abc(spec, y, s2.seed, s2.first_draw, s2.n_draws, P.PPS_EPS_TOP_FRACTION,
                    0.3)["eps_used"]
        out.append((P.make_abc_job(spec, y, s2, P.PPS_EPS_FIXED, eps, capacity=n),
                    (spec, y, s2, P.PPS_EPS_FIXED, eps, n)))
    jobs, meta = mixed_jobs(P, n_jobs=4, seed=13)
    ob = observed()["logistic_S1000"]["y_obs"]
    mixed = []
    for j, m in zip(jobs, meta):
        if m[0] == "pvalue":
            mixed.append((j, m))
        else:
            mode = P.PPS_EPS_TOP_FRACTION if m[0] == "abc_top" else P.PPS_EPS_FIXED
            mixed.append((j, (m[1], ob, m[2], mode, m[3], None if m[0] == "abc_top" else 4000)))
    # interleaved: the scheduler sees the classes in no particular order
    return out[:2] + mixed[:2] + out[2:] + mixed[2:]


def every_model_alone(P, pairs):
    ref = []
    for _, m in pairs:
        if m[0] == "pvalue":
            ob = observed()["logistic_S1000"]
            c, _ = P.prior_pred_pvalue(m[1], 0, P.PPS_LOGNORMAL, [m[3]], m[2], ob["t_obs"])
            ref.append(({"count_ge": int(c[0])}, 0))
            continue
        spec, y, s, mode, arg, cap = m
        ref.append((P.abc(spec, y, s.seed, s.first_draw, s.n_draws, mode, arg, capacity=cap),
                    len(spec["priors"])))
    return ref


def assert_same_n(P, res, ref, n_params, arena):
    if "count_ge" in ref:
        assert res.status == P.PPS_OK and res.count_ge == ref["count_ge"]
        return
    assert res.status == P.PPS_OK
    assert res.abc.n_accepted == ref["n_accepted"] > 0
    assert res.abc.eps_used == ref["eps_used"]
    np.testing.assert_array_equal(np.array(res.abc.mean[:n_params]), ref["mean"][:n_params])
    np.testing.assert_array_equal(np.array(res.abc.var[:n_params]), ref["var"][:n_params])
    idx, th, d = P.records(res, arena, n_params)
    np.testing.assert_array_equal(idx, ref["idx"].cpu().numpy().astype(np.uint64))
    np.testing.assert_array_equal(th, ref["theta"].cpu().numpy())
    np.testing.assert_array_equal(d, ref["dist"].cpu().numpy())


@pytest.mark.parametrize("policy", ["batched", "plain"])
def test_every_model_batched_equals_alone(P, torch, arena, policy):
    """Toggle-switch and tuberculosis ABC jobs in one batch with
    logistic jobs: each job's records, tolerance and moments equal its
    synchronous run (jobs split over epochs, classes mixed within one)."""
    pairs = every_model_jobs(P)
    ref = every_model_alone(P, pairs)
    pol = P.PPS_POLICY_BATCHED if policy == "batched" else P.PPS_POLICY_PLAIN
    res = P.pps_run_batch([j for j, _ in pairs], P.make_server_config(arena, epoch_ms=0.5, policy=pol))
    for r, (f, n_params) in zip(res, ref):
        assert_same_n(P, r, f, n_params, arena)


def test_every_model_served_equals_alone(P, torch, arena):
    pairs = every_model_jobs(P)
    ref = every_model_alone(P, pairs)
    with P.Server(P.make_server_config(arena, epoch_ms=1.0)) as srv:
        ids = [srv.submit(j) for j, _ in pairs]
        deadline = time.time() + 60
        done = {}
        while len(done) < len(ids) and time.time() < deadline:
            for i, jid in enumerate(ids):
                if i not in done:
                    rc, r = srv.poll(jid)
                    if rc != P.PPS_PENDING:
                        done[i] = r
            time.sleep(0.001)
        assert len(done) == len(ids)
        for i, (f, n_params) in enumerate(ref):
            assert_same_n(P, done[i], f, n_params, arena)
            assert srv.release(ids[i]) == P.PPS_OK
        # p-value jobs stay with the logistic SDE and normal-mean models, and
        # GARCH has tallies, not ABC
        garch = W.garch_spec(series_len=100)
        for bad in (P.make_pvalue_job(garch, 0, P.PPS_UNIFORM, 1e-4, P.make_sampling(100, 0, 1), 0.0),
                    P.make_abc_job(garch, observed()["garch_L2000"]["summaries"],
                                   P.make_sampling(100, 0, 1), P.PPS_EPS_TOP_FRACTION, 0.1)):
            with pytest.raises(P.PPSError):
                srv.submit(bad)


def test_server_small_arena_admission(P, torch):
    """An arena that holds about one ABC job: jobs wait for memory, run as
    releases free it, and still equal their results alone."""
    jobs, meta = mixed_jobs(P, n_jobs=6, seed=11)
    ref = alone(P, meta)
    need = max(P.pps_job_arena_bytes(j) for j in jobs)
    small = torch.empty(need + 4096, dtype=torch.uint8, device="cuda")
    cfg = P.make_server_config(small, epoch_ms=1.0)
    with P.Server(cfg) as srv:
        ids = [srv.submit(j) for j in jobs]
        pending = dict(enumerate(ids))
        deadline = time.time() + 60
        while pending and time.time() < deadline:
            for i, jid in list(pending.items()):
                rc, r = srv.poll(jid)
                if rc != P.PPS_PENDING:
                    assert_same(P, r, ref[i], small)
                    assert srv.release(jid) == P.PPS_OK
                    del pending[i]
            time.sleep(0.001)
        assert not pending


def test_server_errors(P, torch):
    ob = observed()["logistic_S1000"]
    spec = W.logistic_spec(steps=200)
    big = P.make_abc_job(spec, ob["y_obs"], P.make_sampling(1_000_000, 0, 1), P.PPS_EPS_TOP_FRACTION, 0.01)
    small = P.make_abc_job(spec, ob["y_obs"], P.make_sampling(2000, 0, 1), P.PPS_EPS_TOP_FRACTION, 0.01)
    arena = torch.empty(P.pps_job_arena_bytes(small) + 256, dtype=torch.uint8, device="cuda")
    # a job larger than the whole arena fails with ENOMEM, the next one runs
    cfg = P.make_server_config(arena, epoch_ms=1.0, queue_capacity=2)
    with P.Server(cfg) as srv:
        jb = srv.submit(big)
        deadline = time.time() + 30
        rc = P.PPS_PENDING
        while rc == P.PPS_PENDING and time.time() < deadline:
            rc, r = srv.poll(jb)
        assert rc == P.PPS_ENOMEM
        # memory held by a finished, unreleased job keeps later jobs queued:
        # the queue fills and submit answers EBUSY
        a = srv.submit(small)
        while srv.poll(a)[0] == P.PPS_PENDING and time.time() < deadline:
            time.sleep(0.001)
        b = srv.submit(small)
        c = srv.submit(small)
        assert srv.try_submit(small) is None  # queue_capacity 2 reached
        assert srv.release(b) == P.PPS_EBUSY  # not finished: cannot release
        assert srv.release(a) == P.PPS_OK     # frees memory: b and c run
        for jid in (b, c):
            while srv.poll(jid)[0] == P.PPS_PENDING and time.time() < deadline:
                time.sleep(0.001)
            assert srv.poll(jid)[0] == P.PPS_OK
            assert srv.release(jid) == P.PPS_OK
        with pytest.raises(P.PPSError):
            srv.poll(12345)


def test_server_error_completes_every_job(P, torch, arena):
    """After an error (injected from the host once two epochs have been
    harvested; the device runs every epoch to its end) the server stops:
    every job that had not finished completes with that error, pps_poll never
    stays PENDING, and later submissions are refused with it."""
    jobs, meta = mixed_jobs(P, n_jobs=24, seed=13)
    ref = alone(P, meta)
    cfg = P.make_server_config(arena, epoch_ms=0.3, max_active=4)
    with P.Server(cfg) as srv:
        srv.inject_error(2, P.PPS_EDEVICE)
        ids = [srv.submit(j) for j in jobs]
        status = {}
        deadline = time.time() + 30
        while len(status) < len(ids) and time.time() < deadline:
            for i, jid in enumerate(ids):
                if i not in status:
                    rc, r = srv.poll(jid)
                    if rc != P.PPS_PENDING:
                        status[i] = rc
                        if rc in (P.PPS_OK, P.PPS_ETRUNC):
                            assert_same(P, r, ref[i], arena)
            time.sleep(0.001)
        assert len(status) == len(ids), "jobs left pending after the error"
        failed = [i for i, rc in status.items() if rc == P.PPS_EDEVICE]
        assert failed and all(rc in (P.PPS_OK, P.PPS_ETRUNC, P.PPS_EDEVICE) for rc in status.values())
        print(f"{len(ids) - len(failed)} jobs finished before the error, {len(failed)} failed with it")
        with pytest.raises(P.PPSError) as e:
            srv.submit(jobs[0])
        assert e.value.status == P.PPS_EDEVICE
        for jid in ids:
            assert srv.release(jid) == P.PPS_OK


def test_server_destroy_drops_backlog(P, torch, arena):
    """Destroying a server with a long backlog waits for the epochs in flight
    only: it returns long before the backlog could have run."""
    ob = observed()["logistic_S1000"]
    spec = W.pvalue_spec(steps=5000)
    job = P.make_pvalue_job(spec, 0, P.PPS_LOGNORMAL, 0.5, P.make_sampling(1_000_000, 0, 1), ob["t_obs"])
    n_jobs = 600  # 3e12 Euler steps: over a second of GPU time
    srv = P.Server(P.make_server_config(arena, epoch_ms=2.0))
    try:
        for _ in range(n_jobs):
            srv.submit(job)
        time.sleep(0.05)
        st = srv.stats()
        assert st.completed < n_jobs
    finally:
        t0 = time.perf_counter()
        srv.close()
        dt = time.perf_counter() - t0
    print(f"destroy with {n_jobs - st.completed} jobs left took {dt * 1e3:.1f} ms")
    assert dt < 0.3


def test_batch_truncation_and_enomem(P, torch, arena):
    ob = observed()["logistic_S1000"]
    spec = W.logistic_spec(steps=200)
    s = P.make_sampling(5000, 0, 3)
    j_fixed = P.make_abc_job(spec, ob["y_obs"], s, P.PPS_EPS_FIXED, 80.0, capacity=5)
    res = P.pps_run_batch([j_fixed], P.make_server_config(arena))
    assert res[0].status == P.PPS_ETRUNC and res[0].n_records == 5 and res[0].abc.n_accepted > 5
    ref = P.abc(spec, ob["y_obs"], 3, 0, 5000, P.PPS_EPS_FIXED, 80.0, capacity=5)
    assert res[0].abc.n_accepted == ref["n_accepted"]
    idx, _, _ = P.records(res[0], arena, 3)
    np.testing.assert_array_equal(idx, ref["idx"].cpu().numpy().astype(np.uint64))
    j_big = P.make_abc_job(spec, ob["y_obs"], P.make_sampling(2_000_000, 0, 3), P.PPS_EPS_TOP_FRACTION, 0.01)
    tiny = arena[: 1 << 20]
    res = P.pps_run_batch([j_big, j_fixed], P.make_server_config(tiny))
    assert res[0].status == P.PPS_ENOMEM and res[1].status == P.PPS_ETRUNC
