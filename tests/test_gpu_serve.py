"""Serving loop on the GPU: results served inside mixed batches equal the same
requests run alone (batch invariance), mixed precision stays within its bar,
graph replay reproduces eager results round after round, and admission under a
small HBM budget evicts plans and still serves every request correctly."""
import numpy as np
import pytest

from .gpu_util import alm_inputs, from_dev, note, rel_rms, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mods():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2208_10154_amd import serve, sht
    sht.lib()
    return serve, sht, torch


def make_request(serve, torch, nside, spin, direction, precision, nmaps, seed):
    lmax = 3 * nside - 1
    ncomp = 1 if spin == 0 else 3
    if direction == "alm2map":
        _, c = alm_inputs(lmax, nmaps, spin == 2, workload=seed)
        inp = to_dev(c.reshape(nmaps, ncomp, -1))
        out = torch.empty((nmaps, ncomp, 12 * nside * nside), dtype=torch.float64, device="cuda")
    else:
        g = torch.Generator(device="cuda")
        g.manual_seed(seed)
        inp = torch.randn((nmaps, ncomp, 12 * nside * nside), generator=g, dtype=torch.float64, device="cuda")
        out = torch.empty((nmaps, ncomp, (lmax + 1) ** 2), dtype=torch.float64, device="cuda")
    return serve.Request(nside=nside, spin=spin, direction=direction, precision=precision, nmaps=nmaps,
                         inp=inp, out=out, arrival=0.0)


def alone(sht, torch, r, precision="fp64"):
    p = sht.Plan(r.nside, r.lmax, r.spin, r.nmaps, precision=precision)
    out = torch.empty_like(r.out)
    (p.alm2map if r.direction == "alm2map" else p.map2alm)(r.inp, out)
    p.sync()
    p.close()
    return from_dev(out)


def mix(serve, torch, precisions=("fp64",), seed0=100):
    reqs, k = [], 0
    rng = np.random.default_rng(seed0)
    for nside in (8, 16):
        for spin in (0, 2):
            for direction in ("alm2map", "map2alm"):
                for prec in precisions:
                    for _ in range(3):
                        reqs.append(make_request(serve, torch, nside, spin, direction, prec,
                                                 int(rng.integers(1, 6)), seed0 + k))
                        k += 1
    return reqs


def test_batch_invariance_fp64(mods):
    serve, sht, torch = mods
    note("serve: batch invariance fp64")
    s = serve.Server(20e9, max_slots=64, executor=serve.Executor(nstreams=2))
    reqs = mix(serve, torch)
    for r in reqs:
        s.submit(r)
    s.drain()
    torch.cuda.synchronize()
    assert max(n for _, _, n, _ in s.batches) > 5  # requests were actually grouped
    for r in reqs:
        assert r.status == 0 and r.latency is not None and r.latency >= 0
        err = rel_rms(from_dev(r.out), alone(sht, torch, r))
        assert np.all(err <= 1e-12), (r.key, err)
    s.close()


def test_mixed_precision_within_bar(mods):
    serve, sht, torch = mods
    note("serve: mixed precision")
    s = serve.Server(20e9, max_slots=64, executor=serve.Executor(nstreams=2))
    reqs = mix(serve, torch, precisions=("fp32", "bf16x3"), seed0=300)
    for r in reqs:
        s.submit(r)
    s.drain()
    torch.cuda.synchronize()
    for r in reqs:
        err = rel_rms(from_dev(r.out), alone(sht, torch, r))
        assert np.all(err <= 1e-5), (r.key, err)
    s.close()


def test_graph_replay_matches_eager(mods):
    serve, sht, torch = mods
    note("serve: graph replay")
    s = serve.Server(20e9, max_slots=64, executor=serve.Executor(nstreams=1, graphs=True))
    a = torch.randn((256, 256), device="cuda")
    for rnd in range(4):
        reqs = [make_request(serve, torch, 16, 2, d, "fp64", 3, 500 + 10 * rnd + i)
                for i, d in enumerate(("alm2map", "map2alm", "alm2map"))]
        for r in reqs:
            s.submit(r)
        s.drain()
        torch.cuda.synchronize()
        a = a @ a.T / 256.0  # eager work between replays
        torch.cuda.synchronize()
        for r in reqs:
            err = rel_rms(from_dev(r.out), alone(sht, torch, r))
            assert np.all(err <= 1e-12), (rnd, r.key, err)
    assert len(s.ex._graphs) >= 2
    s.close()


def test_graph_replay_with_slots_off_the_bucket_grid(mods):
    """40 slots: a batch of 36 map sets falls in the 64-wide bucket, wider than
    the plan; the graph then covers the 40 slots."""
    serve, sht, torch = mods
    note("serve: graph replay, 40 slots")
    s = serve.Server(20e9, max_slots=40, executor=serve.Executor(nstreams=1, graphs=True))
    for rnd in range(2):
        reqs = [make_request(serve, torch, 16, 2, "alm2map", "fp64", 12, 900 + 10 * rnd + i) for i in range(3)]
        for r in reqs:
            s.submit(r)
        s.drain()
        torch.cuda.synchronize()
        for r in reqs:
            assert r.status == 0
            assert np.all(rel_rms(from_dev(r.out), alone(sht, torch, r)) <= 1e-12), (rnd, r.key)
    assert any(b[2] == 36 for b in s.batches)
    s.close()


def test_small_budget_evicts_and_serves(mods):
    serve, sht, torch = mods
    note("serve: small budget")
    need = max(serve.plan_bytes_estimate(n, 3 * n - 1, 2, 64) for n in (8, 16))
    s = serve.Server(1.6 * need, max_slots=64, executor=serve.Executor(nstreams=2))
    reqs = []
    for i in range(6):
        r = make_request(serve, torch, 8 if i % 2 == 0 else 16, 2, "alm2map", "fp64", 2, 700 + i)
        r.arrival = 0.02 * i
        reqs.append(r)
        s.submit(r)
    s.drain()
    torch.cuda.synchronize()
    assert s.peak <= s.budget
    for r in reqs:
        assert r.status == 0
        assert np.all(rel_rms(from_dev(r.out), alone(sht, torch, r)) <= 1e-12)
    s.close()


@pytest.mark.parametrize("nside,spin,slots", [(16, 0, 5), (16, 2, 64), (32, 2, 70), (64, 0, 200)])
def test_footprint_estimate_bounds_the_library(mods, nside, spin, slots):
    serve, sht, torch = mods
    p = sht.Plan(nside, 3 * nside - 1, spin, slots, chunk=serve.bucket(slots))
    actual = p.table_bytes() + p.workspace_bytes()
    p.close()
    est = serve.plan_bytes_estimate(nside, 3 * nside - 1, spin, slots)
    assert actual <= est <= 1.5 * actual + (64 << 20), (actual, est)


def _oracle_request(serve, torch, spin, direction, precision, nmaps, workload):
    """A served request at nside 64 (lmax 191) on seeded inputs, with the oracle's
    result for them: alm2map of Gaussian a_lm, map2alm of white maps."""
    import oracle
    from paper_2208_10154_amd import synth
    nside, lmax, nc = 64, 191, (1 if spin == 0 else 3)
    if direction == "alm2map":
        a, c = alm_inputs(lmax, nmaps, spin == 2, workload=workload)
        ref = oracle.alm2map_iqu(nside, lmax, a) if spin == 2 else oracle.alm2map(nside, lmax, a[:, 0])[:, None]
        inp = to_dev(c)
        out = torch.full((nmaps, nc, 12 * nside * nside), np.nan, dtype=torch.float64, device="cuda")
    else:
        m = synth.white_maps(12 * nside * nside, nmaps, nc, workload=workload)
        ref = oracle.to_compact(oracle.map2alm_iqu(nside, lmax, m) if spin == 2
                                else oracle.map2alm(nside, lmax, m[:, 0])[:, None])
        inp = to_dev(m)
        out = torch.full((nmaps, nc, (lmax + 1) ** 2), np.nan, dtype=torch.float64, device="cuda")
    r = serve.Request(nside=nside, spin=spin, direction=direction, precision=precision, nmaps=nmaps,
                      inp=inp, out=out, arrival=0.0)
    return r, ref


@pytest.mark.parametrize("batching", [True, False])
def test_served_requests_match_the_oracle(mods, batching):
    """One request per key (spin 0 / 2, both directions, FP64 / split BF16) at
    nside 64, served together through the batching server (and through the
    one-request-per-launch baseline), each checked against the oracle: 1e-10
    relative RMS per map and component in FP64, 1e-5 in split BF16."""
    serve, sht, torch = mods
    note(f"serve: served requests against the oracle, batching={batching}")
    kw = dict(executor=serve.Executor(nstreams=2)) if batching else \
        dict(executor=serve.Executor(nstreams=1), batching=False, depth=64)
    s = serve.Server(40e9, max_slots=64, **kw)
    cases, k = [], 0
    for spin in (0, 2):
        for direction in ("alm2map", "map2alm"):
            for prec in ("fp64", "bf16x3"):
                for n in (2, 3):  # two requests per key: batched together when batching
                    cases.append(_oracle_request(serve, torch, spin, direction, prec, n, 810 + k))
                    k += 1
    for r, _ in cases:
        s.submit(r)
    s.drain()
    torch.cuda.synchronize()
    if batching:
        assert any(nr > 1 for _, _, _, nr in s.batches)
    else:
        assert all(nr == 1 for _, _, _, nr in s.batches)
    tol = {"fp64": 1e-10, "bf16x3": 1e-5}
    for r, ref in cases:
        assert r.status == 0
        got = from_dev(r.out)
        assert np.all(np.isfinite(got))
        err = rel_rms(got, ref)
        assert np.all(err <= tol[r.precision]), (r.key, err)
    s.close()
