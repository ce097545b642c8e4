"""The allocation-free entry point bires_resultant_noalloc (through the C ABI)
against the existing entry points bires_resultant / bires_discriminant, bit for
bit, on consecutive calls (each later one on a smaller input), with host- and
device-memory buffers, several reconstruction routes and the size limit."""

import pytest

import paper_1201_1548_amd as br
from oracle.resultant import discriminant_y, resultant_x, resultant_y
from paper_1201_1548_amd import synth
from tests.golden.make_golden import load

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


@pytest.mark.parametrize("device", [False, True])
def test_noalloc_equals_resultant_on_consecutive_calls(device):
    br.init()
    F, G = synth.pair_deg20(0)
    say("noalloc deg20 pair 0, device memory", device)
    ref = br.resultant(F, G)
    assert ref == load("deg20_res_0.txt")[1]
    assert br.resultant_noalloc(F, G, device=device) == ref
    # second call, smaller input: the scratch holds the first call's data
    F6, G6 = synth.pair_deg6(3)
    say("noalloc deg6 pair 3")
    got = br.resultant_noalloc(F6, G6, device=device)
    assert got == br.resultant(F6, G6) == load("deg6_res_3.txt")[1]
    # a third, smaller still, by x
    H, K = synth.random_rect(1500, 3, 2, 2, 3, 40)
    say("noalloc res_x small")
    assert br.resultant_noalloc(H, K, var="x", device=device) == br.resultant(H, K, var="x") == resultant_x(H, K)


@pytest.mark.parametrize("device", [False, True])
def test_noalloc_discriminant_then_smaller(device):
    br.init()
    F = synth.curve_deg40(7, tdeg=14, bits=16)
    say("noalloc discriminant tdeg 14, device memory", device)
    assert br.resultant_noalloc(F, kind="disc", device=device) == br.discriminant(F)
    F2 = synth.curve_deg40(8, tdeg=6, bits=12)
    got = br.resultant_noalloc(F2, kind="disc", device=device)
    assert got == br.discriminant(F2) == discriminant_y(F2)


def test_noalloc_more_than_128_primes_and_special_results():
    br.init()
    F, G = synth.random_rect(1300, 5, 6, 5, 6, 400)
    assert br.plan(F, G)[1] > 128
    say("noalloc with P > 128")
    assert br.resultant_noalloc(F, G) == br.resultant(F, G) == resultant_y(F, G)
    F2, G2 = synth.random_rect(1301, 2, 3, 2, 2, 300)
    assert br.resultant_noalloc(F2, G2, device=True) == br.resultant(F2, G2) == resultant_y(F2, G2)
    say("noalloc special results")
    assert br.resultant_noalloc([[0, 0]], G2, device=True) == []
    assert br.resultant_noalloc([[3, 1]], [[7, 2]], device=True) == [1]
    assert br.resultant_noalloc([[3, 1]], G2) == resultant_y([[3, 1]], G2)


def test_noalloc_rejects_jobs_beyond_the_scratch():
    br.init()
    F, G = synth.random_dense(1600, 64, 128)
    say("noalloc beyond the scratch size")
    with pytest.raises(br.BiresError) as ei:
        br.resultant_noalloc(F, G)
    assert ei.value.code == -4
    # the entry point still works afterwards
    F6, G6 = synth.pair_deg6(1)
    assert br.resultant_noalloc(F6, G6) == load("deg6_res_1.txt")[1]
