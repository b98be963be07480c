"""Pins of the oracle's modulus switching of the reply (a wire-format variant of the sparse
reply of section 3.1.3: the server drops the last RNS prime before sending, so every reply
coefficient crosses the wire with L - 1 residues instead of L).

- brute force on tiny primes: every c in [0, q) maps to the nearest integer to c q'/q, computed
  with exact fractions (a floor instead of the rounding, or the wrong prime dropped, fails);
- closed form: exact multiples of the dropped prime map to their quotient;
- the protocol: decrypting the switched reply (with the first L - 1 primes) gives the same
  client share as the unswitched reply, so the shares still add up to X W, for two and three
  primes and several plans;
- the noise: the switched reply's measured noise stays under noise_bound_switched, and
  switch_ok is the bound's condition (it refuses a plaintext modulus too large for q').
"""
from fractions import Fraction

import numpy as np
import pytest

from paper_2305_18396_amd import workloads


def tiny_params(orc, qs, N=16, ell=4):
    return orc.Params(N, len(qs), ell, 2, q=list(qs), psi=[orc.find_psi(q, N) for q in qs])


def residues(c_values, qs):
    return np.array([[[c % q for c in c_values] for q in qs]], dtype=np.uint64)


@pytest.mark.parametrize("qs", [(97, 193), (97, 193, 449)])
def test_switch_brute_force(orc, qs):
    p = tiny_params(orc, qs)
    Q = int(np.prod([int(q) for q in qs]))
    qd = qs[-1]
    rng = np.random.default_rng(5)
    cs = list(range(min(Q, 20000))) if Q <= 20000 else [int(v) for v in rng.integers(0, Q, 20000)]
    cs += [Q - 1, Q - qd // 2 - 1, Q - qd // 2, qd // 2, qd // 2 + 1]
    got = orc.mod_switch(p, residues(cs, qs))
    qs_prime = Q // qd
    for i, c in enumerate(cs):
        want = round(Fraction(c * qs_prime, Q)) % qs_prime
        for l in range(len(qs) - 1):
            assert int(got[0, l, i]) == want % qs[l], (c, l)


def test_switch_exact_multiples(orc):
    p = orc.Params(4096, 2, 37, 12)
    qd = p.q[-1]
    ks = [0, 1, 2, 12345, p.q[0] - 1]
    got = orc.mod_switch(p, residues([k * qd for k in ks], p.q))
    assert [int(v) for v in got[0, 0]] == [k % p.q[0] for k in ks]


def switched_share(orc, p, plan, res):
    """The client's share decrypted from the switched reply with the first L - 1 primes."""
    ps = orc.switched_params(p)
    c1s = orc.mod_switch(p, res["c1"])
    c0ss = orc.mod_switch(p, res["c0s"])
    return orc.decrypt(ps, plan, res["s"], c1s, c0ss, res["outs"]), ps, c1s, c0ss


@pytest.mark.parametrize("N,L,ell,f,shape,plan_kw", [
    (4096, 2, 37, 12, (16, 64, 64), {}),
    (4096, 2, 37, 12, (40, 300, 200), dict(d_fix=256)),
    (8192, 3, 41, 14, (33, 100, 70), {}),
])
def test_switched_reply_gives_the_same_share(orc, N, L, ell, f, shape, plan_kw):
    n, r, m = shape
    rng = np.random.default_rng(N + n)
    X = workloads.share(rng, n, r, ell)
    W = workloads.weights(rng, r, m, f)
    p = orc.Params(N, L, ell, f)
    plan = (orc.plan_fix(N, plan_kw["d_fix"], n, r, m) if plan_kw else orc.plan_comm(N, n, r, m))
    assert orc.switch_ok(p, plan, int(np.abs(W).max()))
    res = orc.pi_matmul(p, plan, X, W, workloads.seed("client", 81), workloads.seed("server", 81),
                        op_id=81)
    Y0s, ps, c1s, c0ss = switched_share(orc, p, plan, res)
    assert c1s.shape == (plan.O, L - 1, N) and c0ss.shape == (plan.O, L - 1, plan.mb * plan.nb)
    assert np.array_equal(Y0s, res["Y0"])
    Y = (Y0s + res["Y1"]) & np.uint64(p.t - 1)
    Xu, Wu = np.asarray(X, np.uint64), np.asarray(W, np.int64).astype(np.uint64)
    assert np.array_equal(Y, (Xu @ Wu) & np.uint64(p.t - 1))


def test_switched_noise_under_bound(orc):
    """Noise of the switched reply at the decoded positions: [c0' + c1' s]_{q'} minus the
    exact scaled message q' v / t (v the decrypted value), centred mod q', against
    noise_bound_switched."""
    p = orc.Params(4096, 2, 37, 12)
    rng = np.random.default_rng(17)
    n, r, m = 16, 64, 64
    X = workloads.share(rng, n, r, 37)
    W = workloads.weights(rng, r, m, 12)
    plan = orc.plan_comm(4096, n, r, m)
    res = orc.pi_matmul(p, plan, X, W, workloads.seed("client", 82), workloads.seed("server", 82),
                        op_id=82)
    Y0s, ps, c1s, c0ss = switched_share(orc, p, plan, res)
    x = orc.decrypt_residues(ps, plan, res["s"], c1s, c0ss)  # [o][mb*nb][L-1]
    qs = ps.Q
    worst = Fraction(0)
    for o, y in enumerate(res["outs"].tolist()):
        ib, kb = divmod(int(y), plan.K)
        for k in range(plan.nb):
            for i in range(plan.mb):
                row, col = kb * plan.nb + k, ib * plan.mb + i
                if row >= n or col >= m:
                    continue
                mval = (int(Y0s[row, col])) % p.t
                xv = int(x[o, k * plan.mb + i, 0])  # one prime left: the residue is the value
                d = (Fraction(xv) - Fraction(qs * mval, p.t)) % qs
                if d > Fraction(qs, 2):
                    d -= qs
                worst = max(worst, abs(d))
    bound = orc.noise_bound_switched(p, plan, int(np.abs(W).max()))
    assert 0 < worst <= bound, (worst, bound)
    assert 2 * p.t * (bound + 1) < qs


def test_switch_ok_is_the_bound(orc):
    plan = orc.plan_comm(4096, 128, 768, 2304)
    wmax = 400
    ok = orc.Params(4096, 2, 37, 12)
    assert orc.switch_ok(ok, plan, wmax)
    # t = 2^40 with one 50-bit prime left: 2 t (N/2) exceeds q'.
    big_t = orc.Params(4096, 2, 40, 12)
    assert not orc.switch_ok(big_t, plan, wmax)
    # The rule matches its formula.
    for prm in (ok, big_t, orc.Params(8192, 3, 41, 14)):
        Eb = orc.noise_bound_switched(prm, plan, wmax)
        assert orc.switch_ok(prm, plan, wmax) == (2 * prm.t * (Eb + 1) < prm.Q // prm.q[-1])
