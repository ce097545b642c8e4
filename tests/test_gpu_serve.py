"""Serving loop (continuous batching) through the C ABI: every result equals
the oracle's and the single-call result, alone or in a mix of concurrent
requests; admission honours the HBM budget."""

import random
import threading

import pytest

import paper_1201_1548_amd as br
from oracle.resultant import discriminant_y, resultant_y
from paper_1201_1548_amd import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def make_requests(n, seed):
    rng = random.Random(seed)
    reqs = []
    for i in range(n):
        kind = rng.choice(["res", "disc"])
        d = rng.randint(1, 7)
        bits = rng.randint(4, 90)
        F, G = synth.random_dense(9000 + seed * 100 + i, d, bits)
        if kind == "disc" and len(F) < 2:
            kind = "res"
        reqs.append((kind, F, G if kind == "res" else None))
    return reqs


def ref(kind, F, G):
    return discriminant_y(F) if kind == "disc" else resultant_y(F, G)


def test_mix_equals_alone_and_oracle():
    reqs = make_requests(40, 1)
    say("serve mix of", len(reqs))
    with br.Server(hbm_budget_bytes=1 << 30, max_slots=16) as srv:
        tickets = [srv.submit(k, F, G) for k, F, G in reqs]
        outs = [srv.wait(t) for t in tickets]
    for (k, F, G), (R, lat) in zip(reqs, outs):
        assert R == ref(k, F, G)
        alone = br.discriminant(F) if k == "disc" else br.resultant(F, G)
        assert R == alone
        assert lat >= 0.0


def test_concurrent_submitters():
    reqs = make_requests(24, 2)
    results = [None] * len(reqs)
    say("concurrent submitters")
    with br.Server(hbm_budget_bytes=1 << 30, max_slots=8) as srv:
        def client(idx):
            for i in idx:
                k, F, G = reqs[i]
                results[i] = srv.wait(srv.submit(k, F, G))[0]
        th = [threading.Thread(target=client, args=(list(range(j, len(reqs), 3)),)) for j in range(3)]
        for t in th:
            t.start()
        for t in th:
            t.join()
    for (k, F, G), R in zip(reqs, results):
        assert R == ref(k, F, G)


def test_budget_admission():
    F, G = synth.pair_deg6(0)
    say("budget admission")
    # a budget that holds one job at a time still completes every request, in order
    with br.Server(hbm_budget_bytes=3 << 20, max_slots=1) as srv:
        ts = [srv.submit("res", F, G) for _ in range(3)]
        outs = [srv.wait(t)[0] for t in ts]
    assert all(o == resultant_y(F, G) for o in outs)
    # a job larger than the whole budget is refused with ENOMEM
    with br.Server(hbm_budget_bytes=4096, max_slots=4) as srv:
        t = srv.submit("res", F, G)
        with pytest.raises(br.BiresError) as ei:
            srv.wait(t)
        assert ei.value.code == -3


def test_unknown_ticket():
    with br.Server(hbm_budget_bytes=1 << 26, max_slots=2) as srv:
        with pytest.raises(br.BiresError) as ei:
            srv._caps = {12345: (0, 1)}
            srv.wait(12345)
        assert ei.value.code == -7


def test_wait_with_small_buffer_keeps_the_ticket():
    # a too-small output buffer reports the needed sizes and keeps the result;
    # waiting again with a buffer of those sizes returns it
    import ctypes

    import numpy as np
    F, G = synth.pair_deg6(2)
    R = resultant_y(F, G)
    say("small buffer")
    with br.Server(hbm_budget_bytes=1 << 28, max_slots=4) as srv:
        t = srv.submit("res", F, G)
        srv._caps.pop(t)
        small = np.zeros((3, 1), dtype=np.uint32)
        od = br.Upoly(2, 1, small.ctypes.data)
        lat = ctypes.c_double()
        e = br.lib().bires_server_wait(srv.h, t, ctypes.byref(od), -1.0, ctypes.byref(lat))
        assert e == -2
        assert od.degree == len(R) - 1
        need = br.limbs_needed(R)
        assert od.limbs == need
        buf = np.zeros((od.degree + 1, od.limbs), dtype=np.uint32)
        od2 = br.Upoly(od.degree, od.limbs, buf.ctypes.data)
        assert br.lib().bires_server_wait(srv.h, t, ctypes.byref(od2), -1.0, ctypes.byref(lat)) == 0
        assert br.limbs_to_ints(buf[: od2.degree + 1]) == R
        # the ticket is retired once the result was delivered
        assert br.lib().bires_server_wait(srv.h, t, ctypes.byref(od2), -1.0, ctypes.byref(lat)) == -7
