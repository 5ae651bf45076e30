"""GPU parity of the learned proposal against the float64 oracle (oracle/nn.py):
log q, the gradient, Adam, bfloat16 rounding, incremental sampling, and the
Metropolis-Hastings acceptance of whole-lattice moves.

Floating point, so the bar is a tolerance: every kernel computes with the
bfloat16 weights and accumulates in float32, the oracle uses the same
bfloat16 values in float64.  Sums of ~10^3 terms in float32 carry a
relative error of order 1e-6 each, so log q (|log q| ~ 10^2..10^3) is held
to 1e-5 relative plus 1e-3 absolute, gradients to 1e-4 of their largest
component.  Sampling and acceptance decisions compare the same uint32
draws against float thresholds: they agree except where a threshold lies
within float32 error of the draw (about 1e-7 per site), so at most one
sampled configuration in sixteen may differ (none in batches below 16),
log q is compared on every configuration that agrees, and every acceptance
decision must agree."""
import sys

import numpy as np
import pytest

import oracle
from oracle import nn as onn
from paper_2402_06415_amd.workloads import nn_initial_params

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2402_06415_amd as lib  # noqa: E402

C = 16


def say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    lib.load_library()
    yield
    torch.cuda.synchronize()


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _bf16(x):
    """float32 -> bfloat16 (round to nearest even) -> float64, on the CPU by torch."""
    return torch.as_tensor(np.asarray(x, np.float32)).to(torch.bfloat16).to(torch.float64).numpy()


def _configs(B, L, seed):
    return np.random.default_rng(seed).choice(np.array([-1, 1], np.int8), size=(B, L, L))


def _net(L, B, seed=0, scale=1.0):
    p = nn_initial_params(seed, scale)
    return lib.Net(L, B, params=p), p


@pytest.mark.parametrize("L,B,seed", [(8, 8, 1), (5, 3, 2), (32, 16, 3), (33, 3, 5), (64, 4, 4)])
def test_logq_matches_oracle(L, B, seed):
    say(f"logq L={L} B={B}")
    net, p = _net(L, B, seed, scale=1.5)
    assert (net.bf16_params() == _bf16(p)).all(), "bfloat16 rounding differs from torch's"
    s = _configs(B, L, seed + 10)
    got = _host(net.logq(torch.from_numpy(s).cuda()))
    want = onn.logq(_bf16(p), s, C)
    assert np.all(np.abs(got - want) <= 1e-5 * np.abs(want) + 1e-3), (got, want)


@pytest.mark.parametrize("L,B", [(8, 8), (32, 16), (64, 2)])
def test_symmetrised_logq_matches_oracle(L, B):
    say(f"logq_sym L={L}")
    net, p = _net(L, B, 13, scale=1.5)
    s = _configs(B, L, 14)
    got = _host(net.logq(torch.from_numpy(s).cuda(), symmetric=True))
    want = onn.logq_sym(_bf16(p), s, C)
    assert np.all(np.abs(got - want) <= 1e-5 * np.abs(want) + 1e-3), (got, want)
    # the two waves' totals trade places and the combination is symmetric
    neg = _host(net.logq(torch.from_numpy(-s).cuda(), symmetric=True))
    assert (neg == got).all()


@pytest.mark.parametrize("L,B", [(8, 16), (32, 64), (7, 5), (64, 2)])
def test_gradient_matches_oracle(L, B):
    say(f"grad L={L} B={B}")
    net, p = _net(L, B, 5, scale=1.5)
    s = _configs(B, L, 6)
    loss = _host(net.loss_and_grad(torch.from_numpy(s).cuda()))[0]
    lw, gw = onn.loss_and_grad(_bf16(p), s, C)
    g = _host(net.grad)
    assert abs(loss - lw) <= 1e-5 * abs(lw) + 1e-4
    scale = np.abs(gw).max()
    assert np.abs(g - gw).max() <= 1e-4 * scale, np.abs(g - gw).max() / scale


def test_adam_steps_match_oracle():
    say("adam")
    L, B = 8, 16
    net, p = _net(L, B, 7)
    s = torch.from_numpy(_configs(B, L, 8)).cuda()
    master = p.astype(np.float64)
    m = np.zeros_like(master)
    v = np.zeros_like(master)
    for step in range(1, 4):
        net.loss_and_grad(s)
        g = _host(net.grad).astype(np.float64)
        net.adam(1e-2)
        master, m, v = onn.adam_step(master, m, v, g, step, 1e-2, 0.9, 0.999, 1e-8)
        got = _host(net.master)
        assert np.abs(got - master).max() <= 1e-5 * np.abs(master).max()
        # the next step continues from the device's float32 master
        master = got.astype(np.float64)
        m, v = _host(net.adam_m).astype(np.float64), _host(net.adam_v).astype(np.float64)
    assert (net.bf16_params() == _bf16(_host(net.master))).all()


def _oracle_uniforms(B, N, seed, chain0, draw):
    key = (seed & 0xFFFFFFFF, seed >> 32)
    r = np.zeros((B, N), dtype=np.uint32)
    for b in range(B):
        for g in range((N + 3) // 4):
            out = oracle.philox4x32_10((g, chain0 + b, draw, 6), key)
            for k in range(4):
                if 4 * g + k < N:
                    r[b, 4 * g + k] = out[k]
    return r


@pytest.mark.parametrize("L,B,sym", [(6, 16, False), (16, 8, False), (34, 2, False), (64, 8, False),
                                     (6, 32, True), (20, 8, True)])
def test_sampler_matches_oracle(L, B, sym):
    say(f"sample L={L} B={B} symmetric={sym}")
    net, p = _net(L, B, 9, scale=1.5)
    seed, chain0, draw = (3 << 32) | 17, 5, 2
    s, lq = net.sample(B, seed, chain0, draw, symmetric=sym)
    # the sampler's log q is bitwise the teacher-forced evaluation of its output
    lq_eval = _host(net.logq(s, symmetric=sym))
    s, lq = _host(s), _host(lq)
    assert (lq == lq_eval).all()
    r = _oracle_uniforms(B, L * L, seed, chain0, draw)
    so, lqo = onn.sample(_bf16(p), r, L, C)
    if sym:
        key = (seed & 0xFFFFFFFF, seed >> 32)
        flip = np.array([oracle.philox4x32_10((0xFFFFFFFF, chain0 + b, draw, 6), key)[0] >> 31
                         for b in range(B)], dtype=bool)
        assert 0 < flip.sum() < B
        so = np.where(flip[:, None, None], -so, so)
        lqo = onn.logq_sym(_bf16(p), so, C)
    same = [(s[b] == so[b]).all() for b in range(B)]
    # a sample differs only where a float32 threshold lies within rounding
    # of its uint32 draw (about 1e-7 per site): one in sixteen at most
    allowed = B // 16
    assert B - sum(same) <= allowed, f"{B - sum(same)} of {B} samples differ (allowed {allowed})"
    assert sum(same) >= 1
    for b in range(B):
        if same[b]:
            assert abs(lq[b] - lqo[b]) <= 1e-5 * abs(lqo[b]) + 1e-3, (b, lq[b], lqo[b])


@pytest.mark.parametrize("L,B", [(2, 5), (3, 7), (11, 9), (17, 6), (31, 4), (32, 513), (32, 1024)])
@pytest.mark.parametrize("sym", [False, True])
def test_logq_is_the_samplers_bitwise(L, B, sym):
    """log q of sampled configurations, evaluated the whole lattice at a
    time (L <= 32), is bitwise the log q the wavefront sampler returned:
    odd sides (partial tiles and rows), batches above one configuration per
    CU (each workgroup takes several, fetching the next one's spins ahead)."""
    say(f"logq bitwise L={L} B={B} symmetric={sym}")
    net, _ = _net(L, B, 13, scale=1.5)
    s, lq = net.sample(B, (5 << 32) | 3, 11, 4, symmetric=sym)
    lq_eval = _host(net.logq(s, symmetric=sym))
    lq = _host(lq)
    bad = np.flatnonzero(lq != lq_eval)
    assert bad.size == 0, (bad[:5], lq[bad[:5]], lq_eval[bad[:5]])
    assert np.isfinite(lq).all()


@pytest.mark.parametrize("L", [12, 32, 40])
def test_logq_reads_configurations_at_any_stride(L):
    """Configurations spaced by a stride that is not L^2 (and not a multiple
    of 4) give bitwise the log q of the same configurations packed densely,
    in both forms of the evaluation (whole lattice for L <= 32, wavefront
    above)."""
    say(f"logq stride L={L}")
    B, pad = 37, 13
    net, _ = _net(L, B, 21, scale=1.5)
    dense = torch.as_tensor(_configs(B, L, 8), device="cuda")
    big = torch.zeros((B, L * L + pad), dtype=torch.int8, device="cuda")
    big[:, 5:5 + L * L] = dense.reshape(B, L * L)
    view = big.as_strided((B, L, L), (L * L + pad, L, 1), 5)
    for sym in (False, True):
        want = _host(net.logq(dense, symmetric=sym))
        got = _host(net.logq(view, symmetric=sym))
        assert (got == want).all(), (sym, np.flatnonzero(got != want)[:5])


def test_sampler_draws_from_q():
    """Frequencies of the 2^4 configurations of a 2 x 2 lattice over 2^15
    samples agree with q (chi-square, 15 degrees of freedom)."""
    say("sampler frequencies")
    L, B = 2, 32768
    net, p = _net(L, B, 11, scale=2.0)
    s, _ = net.sample(B, 21)
    s = _host(s).reshape(B, 4)
    code = ((s > 0) * np.array([8, 4, 2, 1])).sum(axis=1)
    counts = np.bincount(code, minlength=16)
    states = np.array([[1 if (c >> (3 - k)) & 1 else -1 for k in range(4)] for c in range(16)],
                      dtype=np.int8).reshape(16, 2, 2)
    q = np.exp(onn.logq(_bf16(p), states, C))
    chi2 = ((counts - q * B) ** 2 / (q * B)).sum()
    assert chi2 < 45.0, chi2


def test_mh_acceptance_matches_oracle():
    """Every acceptance decision equals the oracle's for the same energies,
    log q values, betas and draws; accepted lattices are replaced."""
    say("mh")
    L, count, seed = 8, 64, 99
    rng = np.random.default_rng(12)
    b = lib.Batch([L] * count, [0.44] * count, seed=seed, lattice_id0=3, start="random")
    cur = np.stack([_host(b.lattice(j)) for j in range(count)])
    prop = rng.choice(np.array([-1, 1], np.int8), size=(count, L, L))
    lq_cur = rng.normal(-40.0, 3.0, count).astype(np.float32)
    lq_prop = rng.normal(-40.0, 3.0, count).astype(np.float32)
    beta = rng.uniform(0.0, 0.6, count)
    draw = 4
    acc = torch.zeros(count, dtype=torch.int32, device="cuda")
    # device copies held in names until the kernel has run
    prop_d = torch.from_numpy(prop).cuda()
    lqc_d, lqp_d = torch.from_numpy(lq_cur).cuda(), torch.from_numpy(lq_prop).cuda()
    beta_d = torch.from_numpy(beta).cuda()
    lib.ising_batch_mh(b.c, L, prop_d.data_ptr(), L * L, lqc_d.data_ptr(), lqp_d.data_ptr(),
                       beta_d.data_ptr(), draw, acc.data_ptr(),
                       torch.cuda.current_stream().cuda_stream)
    got = _host(acc)
    Ec = np.array([oracle.measure(x)[0] for x in cur])
    Ep = np.array([oracle.measure(x)[0] for x in prop])
    lr = onn.mh_log_ratio(beta, Ec, Ep, lq_cur, lq_prop)
    key = (seed & 0xFFFFFFFF, seed >> 32)
    want = np.array([oracle.philox4x32_10((3 + j, draw, 0, 7), key)[0] <
                     np.exp(min(0.0, lr[j])) * 4294967296.0 for j in range(count)])
    assert 10 < want.sum() < count - 10  # both outcomes occur
    assert (got == want).all()
    for j in range(count):
        assert (_host(b.lattice(j)) == (prop[j] if want[j] else cur[j])).all()
    b.check()


def test_mh_rejects_lattices_of_another_side():
    say("mh shape")
    b = lib.Batch([8, 16], [0.4, 0.4], seed=1, start="cold")
    prop = torch.ones((2, 8, 8), dtype=torch.int8, device="cuda")
    z = torch.zeros(2, dtype=torch.float32, device="cuda")
    be = torch.zeros(2, dtype=torch.float64, device="cuda")
    acc = torch.full((2,), 7, dtype=torch.int32, device="cuda")
    lib.ising_batch_mh(b.c, 8, prop.data_ptr(), 64, z.data_ptr(), z.data_ptr(), be.data_ptr(), 0,
                       acc.data_ptr(), torch.cuda.current_stream().cuda_stream)
    assert _host(acc)[1] == 0
    with pytest.raises(lib.IsingError):
        b.check()


def test_mh_checks_the_batch_itself():
    """The acceptance step validates its batch without a separate prepare
    launch: with the workspace's setup word cleared from the host it changes
    no lattice, reports 0 for every chain and raises the not-set-up error;
    a lattice of the wrong side names the side in the error."""
    say("mh not set up")
    b = lib.Batch([8, 8], [0.4, 0.4], seed=1, start="cold")
    before = _host(b.spins).copy()
    prop = -torch.ones((2, 8, 8), dtype=torch.int8, device="cuda")
    z = torch.zeros(2, dtype=torch.float32, device="cuda")
    be = torch.zeros(2, dtype=torch.float64, device="cuda")  # beta = 0: every move accepted
    acc = torch.full((2,), 7, dtype=torch.int32, device="cuda")
    magic = b.workspace[0:4].clone()
    b.workspace[0:4] = 0
    lib.ising_batch_mh(b.c, 8, prop.data_ptr(), 64, z.data_ptr(), z.data_ptr(), be.data_ptr(), 0,
                       acc.data_ptr(), torch.cuda.current_stream().cuda_stream)
    assert (_host(acc) == 0).all()
    assert (_host(b.spins) == before).all()
    with pytest.raises(lib.IsingError, match="not set up"):
        b.check()
    # restored, the same call accepts both moves
    b.workspace[0:4] = magic
    lib.ising_batch_mh(b.c, 8, prop.data_ptr(), 64, z.data_ptr(), z.data_ptr(), be.data_ptr(), 0,
                       acc.data_ptr(), torch.cuda.current_stream().cuda_stream)
    assert (_host(acc) == 1).all()
    b.check()
    c = lib.Batch([8, 16], [0.4, 0.4], seed=1, start="cold")
    lib.ising_batch_mh(c.c, 8, prop.data_ptr(), 64, z.data_ptr(), z.data_ptr(), be.data_ptr(), 0,
                       acc.data_ptr(), torch.cuda.current_stream().cuda_stream)
    with pytest.raises(lib.IsingError, match="side differs"):
        c.check()
