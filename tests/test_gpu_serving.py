"""Serving: requests submitted to the context's queue are batched into segmented
sorts; every result must be the stable sort of that request alone (the oracle's),
bit for bit, whatever else shares its batch."""
from __future__ import annotations

import time

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available()
    return t


@pytest.fixture(scope="module")
def o():
    return oracle.get()


def make_requests(count, seed, lo=1 << 10, hi=1 << 20, key_only_every=7):
    """(keys, vals or None) host arrays: 70% uint32 / 30% uint64, uniform or Zipf."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n = int(np.floor(np.exp(rng.uniform(np.log(lo), np.log(hi)))))
        bits = 64 if rng.uniform() < 0.3 else 32
        dist = "zipf" if rng.uniform() < 0.5 else "uniform"
        k = workloads.make_keys(dist, n, bits, seed * 1000 + i)
        key_only = key_only_every > 0 and i % key_only_every == 3
        v = None if key_only else workloads.index_payload(n, bits)
        out.append((k, v))
    return out


def wait_all(ctx, tickets, timeout_s=60.0):
    lat = {}
    t_end = time.time() + timeout_s
    while len(lat) < len(tickets):
        for t in tickets:
            if t in lat:
                continue
            done, l = ctx.poll(t)
            if done:
                lat[t] = l
        assert time.time() < t_end, "serving did not finish"
        time.sleep(0.0005)
    return lat


def test_mix_equals_alone(torch, o):
    import paper_2207_14334_amd as dfr
    reqs = make_requests(80, 1)
    reqs.append((np.empty(0, np.uint32), np.empty(0, np.uint32)))
    reqs.append((np.array([7], np.uint64), np.array([0], np.uint64)))
    say("serving mix", len(reqs), sum(k.size for k, _ in reqs))
    with dfr.Context(0) as ctx:
        dev = [(torch.from_numpy(k).cuda(), None if v is None else torch.from_numpy(v).cuda())
               for k, v in reqs]
        torch.cuda.synchronize()
        tickets = [ctx.submit(k, v) for k, v in dev]
        lat = wait_all(ctx, tickets)
        st = ctx.serve_stats()
        assert st["requests"] == len(reqs) and st["batches"] < len(reqs), st
        assert st["max_batch_requests"] > 1, st
        assert all(lat[t] > 0 for t in tickets)
        # Every result is the oracle's sort of that request alone, and the same as a
        # plain call on that request alone.
        for (k, v), (dk, dv) in zip(reqs, dev):
            rk, rv = o.stable_sort(k, v)
            assert np.array_equal(dk.cpu().numpy(), rk)
            if v is not None:
                assert np.array_equal(dv.cpu().numpy(), rv)
        for (k, v), (dk, dv) in list(zip(reqs, dev))[:20]:
            ak = torch.from_numpy(k).cuda()
            av = None if v is None else torch.from_numpy(v).cuda()
            ctx.sort_(ak, av)
            torch.cuda.synchronize()
            assert torch.equal(ak, dk) and (av is None or torch.equal(av, dv))


def test_poll_states_and_errors(torch):
    import paper_2207_14334_amd as dfr
    with dfr.Context(0) as ctx:
        with pytest.raises(dfr.DfrError) as e:
            ctx.poll(12345)
        assert e.value.status == dfr.E_NOT_FOUND
        ctx.set_option("serve_workers", 1)
        ctx.set_option("serve_batch_records", 1 << 20)
        k = torch.from_numpy(np.arange(5000, 0, -1, dtype=np.uint32)).cuda()
        torch.cuda.synchronize()
        t = ctx.submit(k)
        done = False
        for _ in range(20000):
            done, _lat = ctx.poll(t)
            if done:
                break
            time.sleep(0.0005)
        assert done
        assert np.array_equal(k.cpu().numpy(), np.arange(1, 5001, dtype=np.uint32))
        with pytest.raises(dfr.DfrError) as e:
            ctx.poll(t)  # consumed
        assert e.value.status == dfr.E_NOT_FOUND
        with pytest.raises(dfr.DfrError) as e:
            ctx.set_option("serve_workers", 2)  # fixed once serving has started
        assert e.value.status == dfr.E_UNSUPPORTED
        bad = torch.empty(10, dtype=torch.uint64, device="cuda")
        with pytest.raises(dfr.DfrError) as e:
            ctx.submit(k[:10], bad)  # payload width differs from key width
        assert e.value.status == dfr.E_INVALID_ARG


def test_budget_admission(torch, o):
    """A small budget: a request that can never fit is refused; the others all finish,
    in batches that keep the workers' memory within the budget."""
    import paper_2207_14334_amd as dfr
    budget = 160 << 20
    reqs = make_requests(40, 2, lo=1 << 10, hi=1 << 19, key_only_every=0)
    say("serving budget", budget, len(reqs))
    with dfr.Context(0, hbm_budget_bytes=budget) as ctx:
        big = torch.empty(1 << 23, dtype=torch.uint64, device="cuda")
        bigv = torch.empty(1 << 23, dtype=torch.uint64, device="cuda")
        with pytest.raises(dfr.DfrError) as e:
            ctx.submit(big, bigv)
        assert e.value.status == dfr.E_BUDGET
        dev = [(torch.from_numpy(k).cuda(), torch.from_numpy(v).cuda()) for k, v in reqs]
        torch.cuda.synchronize()
        tickets = [ctx.submit(k, v) for k, v in dev]
        wait_all(ctx, tickets)
        st = ctx.serve_stats()
        assert st["requests"] == len(reqs), st
        assert st["peak_held_bytes"] <= budget, st
        for (k, v), (dk, dv) in zip(reqs, dev):
            rk, rv = o.stable_sort(k, v)
            assert np.array_equal(dk.cpu().numpy(), rk) and np.array_equal(dv.cpu().numpy(), rv)


def test_plain_calls_beside_serving(torch, o):
    """Plain sorts on the caller's stream while the workers serve requests."""
    import paper_2207_14334_amd as dfr
    reqs = make_requests(30, 3)
    with dfr.Context(0) as ctx:
        dev = [(torch.from_numpy(k).cuda(), None if v is None else torch.from_numpy(v).cuda())
               for k, v in reqs]
        pk = workloads.make_keys("uniform", (1 << 22) + 9, 32, 77)
        pv = workloads.index_payload(pk.size)
        dpk, dpv = torch.from_numpy(pk).cuda(), torch.from_numpy(pv).cuda()
        torch.cuda.synchronize()
        say("serving beside plain", len(reqs))
        tickets = [ctx.submit(k, v) for k, v in dev]
        ctx.sort_(dpk, dpv)
        torch.cuda.synchronize()
        wait_all(ctx, tickets)
        rk, rv = o.stable_sort(pk, pv)
        assert np.array_equal(dpk.cpu().numpy(), rk) and np.array_equal(dpv.cpu().numpy(), rv)
        for (k, v), (dk, dv) in zip(reqs, dev):
            rk, rv = o.stable_sort(k, v)
            assert np.array_equal(dk.cpu().numpy(), rk)
            if v is not None:
                assert np.array_equal(dv.cpu().numpy(), rv)


def test_mix_at_full_request_sizes(torch, o):
    """Requests of the serving workload's full size range, log-uniform in [2^10, 2^24],
    with requests of exactly the default batch limit (2^25 records) and one past it (a
    batch of its own, sorted in place), all queued at once; each result is the oracle's
    (checked by the properties that single out the stable sort under the index payload,
    and the rank formula at a sampled place)."""
    import paper_2207_14334_amd as dfr
    reqs = make_requests(24, 5, lo=1 << 10, hi=1 << 24, key_only_every=0)
    for extra, bits in (((1 << 25), 32), ((1 << 25) + 1, 32), ((1 << 24), 64)):
        reqs.append((workloads.make_keys("uniform", extra, bits, extra + bits),
                     workloads.index_payload(extra, bits)))
    say("serving full sizes", len(reqs), sum(k.size for k, _ in reqs))
    with dfr.Context(0) as ctx:
        dev = [(torch.from_numpy(k).cuda(), torch.from_numpy(v).cuda()) for k, v in reqs]
        torch.cuda.synchronize()
        tickets = [ctx.submit(k, v) for k, v in dev]
        wait_all(ctx, tickets, timeout_s=120.0)
        st = ctx.serve_stats()
        assert st["requests"] == len(reqs), st
        rng = np.random.default_rng(5)
        for (k, v), (dk, dv) in zip(reqs, dev):
            ok, ov = dk.cpu().numpy(), dv.cpu().numpy()
            assert o.check_index_payload(k, ok, ov) is None, k.size
            p = int(rng.integers(0, k.size))
            assert o.rank_of(k, int(ov[p])) == p, (k.size, p)


@pytest.mark.gpu
def test_failed_batch_waits_for_its_work(torch, o):
    """A batch reported failed (forced from the host by the serve_fail_batches test hook,
    after the batch's device work is queued) has finished that work before its requests
    are done: the lone request, sorted in place, is already sorted and stays unchanged
    once dfr_poll reports the failure, and the next request is served normally."""
    import paper_2207_14334_amd as dfr
    n = (1 << 22) + 3
    kh = workloads.make_keys("uniform", n, 32, 11)
    want = o.stable_sort(kh)[0]
    with dfr.Context(0) as ctx:
        ctx.set_option("serve_workers", 1)
        ctx.set_option("serve_fail_batches", 1)
        k = torch.from_numpy(kh.copy()).cuda()
        torch.cuda.synchronize()
        t = ctx.submit(k)
        status = None
        for _ in range(40000):
            try:
                done, _lat = ctx.poll(t)
            except dfr.DfrError as e:
                status = e.status
                break
            assert not done, "the injected failure was not reported"
            time.sleep(0.0005)
        assert status == dfr.E_HIP
        first = k.cpu().numpy()
        assert np.array_equal(first, want)
        time.sleep(0.05)
        assert np.array_equal(k.cpu().numpy(), first)
        k2 = torch.from_numpy(kh.copy()).cuda()
        torch.cuda.synchronize()
        t2 = ctx.submit(k2)
        done = False
        for _ in range(40000):
            done, _lat = ctx.poll(t2)
            if done:
                break
            time.sleep(0.0005)
        assert done
        assert np.array_equal(k2.cpu().numpy(), want)
