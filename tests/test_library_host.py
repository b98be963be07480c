"""CPU checks of libpimm: it loads, exports every function include/pimm.h declares,
and its host-side logic (prime rule, error-sampler table, block plan, noise
check, argument validation) agrees with the oracle.  No kernel runs here."""
import itertools
import os
import re

import numpy as np
import pytest

from paper_2305_18396_amd import pimm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    names = set()
    for h in ("pimm.h", "pimm_probe.h"):
        text = open(os.path.join(ROOT, "include", h)).read()
        names |= set(re.findall(r"^\s*(?:const\s+)?\w+[\s\*]+(pimm_\w+)\(", text, re.M))
    return sorted(names)


def test_exports_every_declared_function():
    declared = header_functions()
    assert len(declared) >= 20
    assert sorted(pimm.EXPORTS) == declared
    lib = pimm.lib()
    for name in declared:
        assert hasattr(lib, name), name


@pytest.mark.parametrize("N,L", [(4096, 1), (4096, 2), (8192, 3), (8192, 4)])
def test_primes_match_oracle(orc, N, L):
    assert pimm.params_primes(pimm.make_params(N, L, 37, 12)) == orc.find_primes(N, L)


def test_cdt_matches_oracle(orc):
    assert pimm.cdt() == orc.cdt_table()


SHAPES = [(16, 64, 64), (128, 768, 2304), (128, 768, 768), (128, 768, 3072), (128, 3072, 768),
          (512, 1024, 3072), (512, 4096, 1024), (1, 1, 1), (19, 23, 13), (7, 4096, 3),
          (513, 100, 5000), (37, 768, 768)]


@pytest.mark.parametrize("N", [4096, 8192])
def test_plan_rule_matches_oracle(orc, N):
    prm = pimm.make_params(N, 2, 37, 12)
    for n, r, m in SHAPES:
        got = pimm.plan_rule(prm, n, r, m)
        want = orc.plan_comm(N, n, r, m)
        assert (got.mb, got.rb, got.nb) == (want.mb, want.rb, want.nb), (n, r, m)
        assert (got.M, got.R, got.K, got.I, got.O, got.Wb, got.P) == \
            (want.M, want.R, want.K, want.I, want.O, want.Wb, want.P)
        for D in (16, 32, 256, 1024, N):
            got = pimm.plan_rule(prm, n, r, m, d_fix=D)
            want = orc.plan_fix(N, D, n, r, m)
            assert (got.mb, got.rb, got.nb) == (want.mb, want.rb, want.nb), (n, r, m, D)


def test_plan_sizes():
    prm = pimm.make_params(4096, 2, 37, 12)
    f = pimm.plan_rule(prm, 128, 768, 2304)
    assert (f.mb, f.rb, f.nb, f.I, f.O, f.Wb) == (8, 4, 128, 192, 288, 55296)
    assert f.ct_bytes == 192 * 2 * 2 * 4096 * 8
    assert f.c0s_bytes == 288 * 2 * 8 * 128 * 8
    assert f.weights_bytes == 55296 * 2 * 4096 * 8
    e = pimm.plan_rule(prm, 5, 6, 7, mb=2, rb=3, nb=4)
    assert (e.M, e.R, e.K) == (4, 2, 2)


def test_noise_check_matches_oracle(orc):
    for rr in (True, False):
        prm = pimm.make_params(4096, 2, 37, 12, rr)
        op = orc.Params(4096, 2, 37, 12, rerandomize=rr)
        for (n, r, m) in SHAPES[:7]:
            info = pimm.plan_rule(prm, n, r, m)
            plan = orc.plan_comm(4096, n, r, m)
            for wmax in (0, 1, 300, 600, 5000, 10**5, 2**20, 2**30):
                assert pimm.noise_ok(prm, info, wmax) == orc.noise_ok(op, plan, wmax), \
                    (rr, n, r, m, wmax)
    # Config with three primes: a much larger budget.
    prm3 = pimm.make_params(8192, 3, 41, 14)
    op3 = orc.Params(8192, 3, 41, 14)
    info = pimm.plan_rule(prm3, 512, 4096, 1024, d_fix=1024)
    plan = orc.plan_fix(8192, 1024, 512, 4096, 1024)
    for wmax in (2000, 2**30, 2**40, 2**50):
        assert pimm.noise_ok(prm3, info, wmax) == orc.noise_ok(op3, plan, wmax)


def _switch_edge(orc, op, plan):
    """The largest wmax the oracle's switch rule accepts (bisection; it is monotone in wmax)."""
    lo, hi = 0, 1 << 48
    if not orc.switch_ok(op, plan, lo):
        return -1
    while hi - lo > 1:
        mid = (lo + hi) // 2
        lo, hi = (mid, hi) if orc.switch_ok(op, plan, mid) else (lo, mid)
    return lo


@pytest.mark.parametrize("N,L,ell,f,shape,d", [
    (4096, 2, 37, 12, (128, 768, 768), 0), (4096, 2, 37, 12, (128, 768, 3072), 64),
    (4096, 2, 44, 12, (16, 64, 64), 0), (8192, 3, 41, 14, (512, 4096, 1024), 1024),
    (8192, 3, 48, 14, (512, 4096, 1024), 1024),
    (8192, 4, 41, 14, (512, 1024, 4096), 0)])
def test_switch_check_matches_oracle(orc, N, L, ell, f, shape, d):
    for rr in (True, False):
        prm = pimm.make_params(N, L, ell, f, rr)
        op = orc.Params(N, L, ell, f, rerandomize=rr)
        info = pimm.plan_rule(prm, *shape, d_fix=d)
        plan = orc.plan_fix(N, d, *shape) if d else orc.plan_comm(N, *shape)
        edge = _switch_edge(orc, op, plan)
        for wmax in {0, 1, 600, 2**20, 2**40, max(edge, 0), edge + 1}:
            assert pimm.switch_ok(prm, info, wmax) == orc.switch_ok(op, plan, wmax), (rr, wmax, edge)


def test_switch_check_refuses_one_prime():
    prm = pimm.make_params(4096, 1, 20, 8)
    info = pimm.plan_rule(prm, 16, 64, 64)
    with pytest.raises(pimm.PimmError, match="PIMM_E_UNSUPPORTED"):
        pimm.switch_ok(prm, info, 1)


@pytest.mark.parametrize("bad,code", [
    (dict(N=1000), "PIMM_E_PARAMS"), (dict(N=2048), "PIMM_E_PARAMS"), (dict(L=0), "PIMM_E_PARAMS"),
    (dict(L=5), "PIMM_E_PARAMS"), (dict(log2_t=1), "PIMM_E_PARAMS"),
    (dict(log2_t=49), "PIMM_E_PARAMS")])
def test_bad_params_rejected(bad, code):
    kw = dict(N=4096, L=2, log2_t=37, frac_bits=12)
    kw.update(bad)
    with pytest.raises(pimm.PimmError, match=code):
        pimm.params_primes(pimm.make_params(**kw))


def test_bad_plans_rejected():
    prm = pimm.make_params(4096, 2, 37, 12)
    with pytest.raises(pimm.PimmError, match="PIMM_E_SHAPE"):
        pimm.plan_rule(prm, 0, 4, 4)
    with pytest.raises(pimm.PimmError, match="PIMM_E_SHAPE"):
        pimm.plan_rule(prm, 4, 4, 4, mb=64, rb=64, nb=2)
    with pytest.raises(pimm.PimmError, match="PIMM_E_SHAPE"):
        pimm.plan_rule(prm, 4, 4, 4, d_fix=48)


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    monkeypatch.setattr(pimm, "_lib", None)
    monkeypatch.setattr(pimm, "LIB_PATH", str(tmp_path / "absent.so"))
    with pytest.raises(ImportError, match="not built"):
        pimm.lib()


def test_probe_rejects_bad_arguments():
    """pimm_probe validates its arguments before touching a device."""
    import ctypes
    rate = ctypes.c_double()
    lib = pimm.lib()
    assert lib.pimm_probe(0, 99, 1 << 26, 1, ctypes.byref(rate)) == -1       # kind
    assert lib.pimm_probe(0, pimm.PROBE_READ, 1000, 1, ctypes.byref(rate)) == -1  # too small
    assert lib.pimm_probe(0, pimm.PROBE_FMA64, 10, 1, ctypes.byref(rate)) == -1   # chain too short
    assert lib.pimm_probe(0, pimm.PROBE_READ, 1 << 26, 0, ctypes.byref(rate)) == -1  # reps
    assert lib.pimm_probe(0, pimm.PROBE_READ, 1 << 26, 1, None) == -1


def test_new_entry_points_reject_null_arguments():
    """The FC completion, the seed-compressed upload, the encoding encryption and the in-place
    weight update check their pointers before touching a device."""
    import ctypes
    lib = pimm.lib()
    seed = ctypes.create_string_buffer(32)
    assert lib.pimm_fc_complete(None, None, None, None, None, None, 0, None) == -1
    assert b"pimm_fc_complete" in lib.pimm_last_error()
    assert lib.pimm_encrypt_seeded(None, None, seed, seed, 0, None, None, None, 0, None) == -1
    assert lib.pimm_encrypt_input(None, None, seed, 0, None, None, None, 0, None) == -1
    assert b"pimm_encrypt_input" in lib.pimm_last_error()
    assert lib.pimm_ct_expand(None, seed, 0, None, None, None) == -1
    assert b"pimm_ct_expand" in lib.pimm_last_error()
    assert lib.pimm_weights_update(None, None, 0, None) == -1
    assert b"pimm_weights_update" in lib.pimm_last_error()
