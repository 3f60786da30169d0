"""GPU parity of direct (autoregressive) sampling (Appendix A, Eqs. A2-A7)
through the C ABI, against the oracle's sampler on the same seeded inputs.

Bars: drawn configurations bit-exact for every chain whose uniforms all stay
1e-9 away from a running sum of its conditionals (the oracle reports that
distance); log p within 1e-10 relative; the dynamic diagonal weight within
1e-14; importance weights within 1e-9 relative.  With boundaries that
truncate nothing the draws are exact, which is checked by a chi^2 test
against |rho|^2 / Z and by importance weights that are all equal.
"""
import math
import sys

import numpy as np
import pytest

import synth
from oracle import direct, measure, network
from oracle.lattice import MODEL_HUBBARD, Lattice

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

TIE = 1e-9


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    return torch.device("cuda:0")


def _say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def _compare(lat, th, chi, chi_dl, seed, draw, cfg, lp, reweight=False, b_diag=1.0, chains=None):
    bdl = direct.double_layer_bottoms(lat, th, chi_dl)
    compared = 0
    for ch in (range(cfg.shape[0]) if chains is None else chains):
        r = direct.sample(lat, th, chi, chi_dl, seed, ch, draw, reweight=reweight, b_diag=b_diag, bdl=bdl)
        if r["gap"] < TIE:
            print("near-tie, chain", ch, r["gap"], flush=True)
            continue
        compared += 1
        assert np.array_equal(cfg[ch], r["S"].astype(np.uint8)), (ch, cfg[ch], r["S"])
        assert abs(lp[ch] - r["log_p"]) <= 1e-10 * max(1.0, abs(r["log_p"])), (ch, lp[ch], r["log_p"])
    return compared


def test_direct_p2_matches_oracle_4x4():
    """4x4 Heisenberg, D = 2, chi = 4, chi_dl = 16 (the double layer's
    bottom boundaries truncate), random unit tensors, 64 chains."""
    import paper_2409_05285_amd as p
    dev = _dev()
    _say("direct p2 4x4 D2 chi4 chi_dl16")
    L1 = L2 = 4
    desc = p.Desc(L1, L2, 2, 4)
    th = synth.theta_random_unit(L1, L2, 2, 2, seed=91)
    cfg, lp, st = p.peps_direct_sample(desc, torch.tensor(th, device=dev), 64, 16, seed=31, draw=5)
    torch.cuda.synchronize()
    assert p.check(st) == 0
    lat = Lattice(L1, L2, D=2, chi=4)
    n = _compare(lat, th, 4, 16, 31, 5, cfg.cpu().numpy(), lp.cpu().numpy())
    assert n >= 61


def test_direct_p4_ragged_lattice_and_b_update():
    """3x5 (odd width), D = 2, chi = 3, chi_dl = 6 (both truncating, tile
    edges ragged), reweighted draws with b = 0.4 and the update of b after
    the draw; then a second draw with the updated b."""
    import paper_2409_05285_amd as p
    dev = _dev()
    _say("direct p4 3x5 D2 chi3 chi_dl6")
    L1, L2, D, chi, chi_dl = 3, 5, 2, 3, 6
    desc = p.Desc(L1, L2, D, chi)
    th = synth.theta_random_unit(L1, L2, D, 2, seed=92)
    theta = torch.tensor(th, device=dev)
    b = torch.tensor([0.4], dtype=torch.float64, device=dev)
    lat = Lattice(L1, L2, D=D, chi=chi)
    b_host = 0.4
    for draw in (0, 1):
        cfg, lp, st = p.peps_direct_sample(desc, theta, 48, chi_dl, seed=37, draw=draw, reweight=True, b_diag=b,
                                           update_b=True)
        torch.cuda.synchronize()
        assert p.check(st) == 0
        cfg_h, lp_h = cfg.cpu().numpy(), lp.cpu().numpy()
        n = _compare(lat, th, chi, chi_dl, 37, draw, cfg_h, lp_h, reweight=True, b_diag=b_host)
        assert n >= 45
        b_host = direct.update_b(lat, b_host, cfg_h.astype(np.int64))
        assert abs(b.item() - b_host) <= 1e-14 * b_host, (b.item(), b_host)


def test_direct_importance_weights_match_oracle():
    """Eq. A7 weights from the device log|rho| of the drawn samples and the
    device log p, against the oracle's amplitudes and log p."""
    import paper_2409_05285_amd as p
    dev = _dev()
    _say("direct importance weights 3x4")
    L1, L2, D, chi, chi_dl = 3, 4, 2, 4, 4
    desc = p.Desc(L1, L2, D, chi)
    th = synth.theta_random_unit(L1, L2, D, 2, seed=93)
    theta = torch.tensor(th, device=dev)
    b = torch.tensor([0.5], dtype=torch.float64, device=dev)
    cfg, lp, st = p.peps_direct_sample(desc, theta, 16, chi_dl, seed=41, reweight=True, b_diag=b)
    la, _, _, st2 = p.peps_eval_batch(desc, theta, cfg, want_e=False)
    w = p.peps_importance_weights(la, lp)
    torch.cuda.synchronize()
    assert p.check(st) == 0 and p.check(st2) == 0
    lat = Lattice(L1, L2, D=D, chi=chi)
    bdl = direct.double_layer_bottoms(lat, th, chi_dl)
    lr = []
    for S in cfg.cpu().numpy().astype(np.int64):
        m = measure.evaluate(lat, th, S, chi, want_O=False)
        lr.append(2.0 * m["log_abs"] - direct.log_prob(lat, th, S, chi, chi_dl, reweight=True, b_diag=0.5, bdl=bdl))
    lr = np.array(lr)
    want = np.exp(lr - lr.max())
    got = w.cpu().numpy()
    assert np.all(np.abs(got - want) <= 1e-9 * want), (got, want)
    assert got.max() == 1.0


def test_direct_hubbard_parity_even_draws():
    """Fermion sampler: 3x3 Hubbard, d^2 = 16, parity-even tensors, D = 2,
    chi = 4, chi_dl = 16, reweighted (b = 0.5): draws against the oracle on
    32 chains, and all 256 drawn configurations of even total parity."""
    import paper_2409_05285_amd as p
    dev = _dev()
    _say("direct hubbard 3x3 d2=16")
    L1 = L2 = 3
    desc = p.Desc(L1, L2, 2, 4, d=4, model=p.MODEL_HUBBARD, t=1.0, U=8.0, mu=4.0, fermionic=1)
    th = synth.theta_random_parity_even(L1, L2, 2, 4, seed=94)
    b = torch.tensor([0.5], dtype=torch.float64, device=dev)
    cfg, lp, st = p.peps_direct_sample(desc, torch.tensor(th, device=dev), 256, 16, seed=43, reweight=True, b_diag=b)
    torch.cuda.synchronize()
    assert p.check(st) == 0
    cfg_h = cfg.cpu().numpy()
    par = np.array([[bin(int(x)).count("1") for x in row] for row in cfg_h]).sum(axis=1) % 2
    assert np.all(par == 0)
    lat = Lattice(L1, L2, D=2, chi=4, d=4, model=MODEL_HUBBARD, t=1.0, U=8.0, mu=4.0)
    n = _compare(lat, th, 4, 16, 43, 0, cfg_h, lp.cpu().numpy(), reweight=True, b_diag=0.5, chains=range(32))
    assert n >= 30


def test_direct_exact_draws_2x2():
    """2x2, D = 2, chi = 4, chi_dl = 16 truncate nothing, so p_2 = |rho|^2/Z:
    4096 device draws pass a chi^2 test against the exact distribution, every
    log p equals log(|rho|^2 / Z), and the importance weights are all 1."""
    import paper_2409_05285_amd as p
    dev = _dev()
    _say("direct exact 2x2, 4096 draws")
    desc = p.Desc(2, 2, 2, 4)
    th = synth.theta_random_unit(2, 2, 2, 2, seed=95)
    theta = torch.tensor(th, device=dev)
    n = 4096
    cfg, lp, st = p.peps_direct_sample(desc, theta, n, 16, seed=47)
    la, _, _, st2 = p.peps_eval_batch(desc, theta, cfg, want_e=False)
    w = p.peps_importance_weights(la, lp)
    torch.cuda.synchronize()
    assert p.check(st) == 0 and p.check(st2) == 0
    lat = Lattice(2, 2, D=2, chi=4)
    cfgs = network.all_configs(lat)
    pr = np.array([network.amplitude(lat, th, S) ** 2 for S in cfgs])
    pr /= pr.sum()
    index = {tuple(S): k for k, S in enumerate(cfgs)}
    ks = np.array([index[tuple(S)] for S in cfg.cpu().numpy().astype(np.int64)])
    lp_h = lp.cpu().numpy()
    assert np.all(np.abs(lp_h - np.log(pr[ks])) <= 1e-10 * np.maximum(1.0, np.abs(lp_h)))
    counts = np.bincount(ks, minlength=len(cfgs)).astype(float)
    exp_ = pr * n
    mask = exp_ > 5
    chi2 = float((((counts - exp_) ** 2)[mask] / exp_[mask]).sum())
    dof = int(mask.sum()) - 1
    assert chi2 < dof + 4.0 * math.sqrt(2 * dof) + 10, (chi2, dof)
    assert np.all(np.abs(w.cpu().numpy() - 1.0) <= 1e-9)


def test_direct_degenerate_calls():
    """n = 0 enqueues nothing; a second call on the same workspace with fewer
    chains gives the same draws for those chains (draws do not depend on the
    batch)."""
    import paper_2409_05285_amd as p
    dev = _dev()
    _say("direct degenerate calls")
    desc = p.Desc(3, 3, 2, 4)
    th = synth.theta_random_unit(3, 3, 2, 2, seed=96)
    theta = torch.tensor(th, device=dev)
    cfg0, lp0, st0 = p.peps_direct_sample(desc, theta, 0, 16, seed=3)
    assert cfg0.shape == (0, 9)
    a, la_, st = p.peps_direct_sample(desc, theta, 40, 16, seed=3, draw=2)
    b, lb_, st2 = p.peps_direct_sample(desc, theta, 7, 16, seed=3, draw=2)
    torch.cuda.synchronize()
    assert p.check(st) == 0 and p.check(st2) == 0
    assert torch.equal(a[:7], b)
    assert torch.equal(la_[:7], lb_)


def test_direct_reuse_double_layer_is_bit_identical():
    """reuse_double_layer: draws on a workspace whose double layer an earlier
    call with the same theta built (and with another number of chains) are
    bit-identical to draws that build it themselves."""
    import paper_2409_05285_amd as p
    dev = _dev()
    _say("direct reuse of the double layer, 4x3 D=2 chi=4 chi_dl=9")
    desc = p.Desc(4, 3, 2, 4)
    th = synth.theta_random_unit(4, 3, 2, 2, seed=97)
    theta = torch.tensor(th, device=dev)
    ws = torch.empty(p.peps_direct_workspace_bytes(desc, 64, 9), dtype=torch.uint8, device=dev)
    b1 = torch.tensor([0.6], dtype=torch.float64, device=dev)
    b2 = b1.clone()
    p.peps_direct_sample(desc, theta, 64, 9, seed=5, draw=0, ws=ws)
    for n, draw in ((23, 1), (64, 2)):
        a, la_, st = p.peps_direct_sample(desc, theta, n, 9, seed=5, draw=draw, reweight=True, b_diag=b1,
                                          update_b=True, reuse_double_layer=True, ws=ws)
        b, lb_, st2 = p.peps_direct_sample(desc, theta, n, 9, seed=5, draw=draw, reweight=True, b_diag=b2,
                                           update_b=True)
        torch.cuda.synchronize()
        assert p.check(st) == 0 and p.check(st2) == 0
        assert torch.equal(a, b) and torch.equal(la_, lb_)
        assert torch.equal(b1, b2)
    with pytest.raises(ValueError):
        p.peps_direct_sample(desc, theta, 4, 9, seed=5, reuse_double_layer=True)


def test_direct_sampling_cooling_2x2_matches_ed():
    """The cooling loop with direct sampling (Appendix A): p_4 draws with the
    dynamic diagonal weight, Eq. A7 importance weights in every average and
    in the SR metric, on 2x2 Heisenberg (D = 4 represents every operator of
    four spins on this ring; chi = 4 and chi_dl = 16 truncate nothing), from
    the identity plus N(0, 0.05^2), 256 chains x 25 draws per step, tau =
    0.01, 25 steps: E/N against exact diagonalisation at beta_phys = 4 n tau
    within 3 sigma + 0.02 |E_ED| at every step, and the diagonal weight
    driven below 1.  The same run with plain p_2 draws (no reweighting) lags
    far behind (the off-diagonal configurations that carry the gradient at
    high temperature are almost never drawn), which is why the reweighting
    exists: at beta_phys = 1 its energy is more than 10 sigma above ED."""
    import paper_2409_05285_amd as p
    from oracle import ed, hamiltonian
    dev = _dev()
    L1 = L2 = 2
    N = L1 * L2
    desc = p.Desc(L1, L2, 4, 4)
    evals = np.linalg.eigvalsh(hamiltonian.dense_H(Lattice(L1, L2, D=1, chi=1)))

    def run(reweight):
        theta = torch.tensor(synth.theta_identity(L1, L2, 4, 2, noise=0.05, seed=97), device=dev)
        configs = torch.tensor(synth.configs_diagonal(256, N, 2, seed=97), device=dev)
        return p.cool(desc, theta, configs, 26, 25, 0.01, 1e-4, 515, cg_iters=200, sampler="direct", chi_dl=16,
                      reweight=reweight)

    _say("direct-sampling cooling 2x2 vs ED, p_4")
    recs = run(True)
    worst = 0.0
    for r in recs:
        e_ed = float(ed.thermal_energy(evals, r["beta_phys"])[0]) / N
        bar = 3 * r["E_stderr"] + 0.02 * abs(e_ed)
        worst = max(worst, abs(r["E_per_site"] - e_ed) / bar)
        print(f"[cool] step {r['step']} beta {r['beta_phys']:.2f} E/N {r['E_per_site']:.5f} +- {r['E_stderr']:.5f} "
              f"ED {e_ed:.5f} b_diag {r['b_diag']:.3f}", flush=True)
        assert r["sampler"] == "direct" and r["accepted_per_sweep"] is None
        assert abs(r["E_per_site"] - e_ed) <= bar, (r["step"], r["E_per_site"], e_ed, bar)
    print("[cool] worst deviation / bar", worst, flush=True)
    assert recs[-1]["b_diag"] < 1.0
    _say("direct-sampling cooling 2x2, plain p_2")
    last = run(False)[-1]
    e_ed = float(ed.thermal_energy(evals, last["beta_phys"])[0]) / N
    print(f"[cool] p_2 at beta {last['beta_phys']:.2f}: E/N {last['E_per_site']:.5f} +- {last['E_stderr']:.5f} "
          f"ED {e_ed:.5f}", flush=True)
    assert last["E_per_site"] - e_ed > 10 * last["E_stderr"]


def test_direct_product_state_closed_form_and_tiny_chi_dl():
    """D = 1 (a product state, 3x4): the conditionals are the single-site
    distributions T_i[x]^2 / sum_x T_i[x]^2 (p_2) or b(x) |T_i[x]| normalised
    (p_4), so log p has a closed form; draws against the oracle.  Then the
    smallest double-layer boundary, chi_dl = 1, on 3x3 D = 2 (every
    double-layer bond truncated to one value): draws and log p against the
    oracle, all finite."""
    import paper_2409_05285_amd as p
    dev = _dev()
    _say("direct D=1 closed form, chi_dl=1")
    L1, L2 = 3, 4
    desc = p.Desc(L1, L2, 1, 1)
    th = synth.theta_random_unit(L1, L2, 1, 2, seed=98)
    lat = Lattice(L1, L2, D=1, chi=1)
    for reweight, bd in ((False, 1.0), (True, 0.3)):
        b = torch.tensor([bd], dtype=torch.float64, device=dev)
        cfg, lp, st = p.peps_direct_sample(desc, torch.tensor(th, device=dev), 40, 1, seed=51, reweight=reweight,
                                           b_diag=b)
        torch.cuda.synchronize()
        assert p.check(st) == 0
        cfg_h, lp_h = cfg.cpu().numpy().astype(np.int64), lp.cpu().numpy()
        for ch in range(40):
            want = 0.0
            for i in range(lat.N):
                t = lat.site_tensor(th, i // L2, i % L2).reshape(4)
                q = t * t / (t * t).sum()
                if reweight:
                    w = np.array([1.0 if x // 2 != x % 2 else bd for x in range(4)]) * np.sqrt(q)
                    q = w / w.sum()
                want += math.log(q[cfg_h[ch, i]])
            assert abs(lp_h[ch] - want) <= 1e-12 * max(1.0, abs(want)), (ch, lp_h[ch], want)
        n = _compare(lat, th, 1, 1, 51, 0, cfg.cpu().numpy(), lp_h, reweight=reweight, b_diag=bd)
        assert n >= 38
    desc = p.Desc(3, 3, 2, 4)
    th = synth.theta_random_unit(3, 3, 2, 2, seed=99)
    cfg, lp, st = p.peps_direct_sample(desc, torch.tensor(th, device=dev), 32, 1, seed=53)
    torch.cuda.synchronize()
    assert p.check(st) == 0
    assert np.all(np.isfinite(lp.cpu().numpy()))
    n = _compare(Lattice(3, 3, D=2, chi=4), th, 4, 1, 53, 0, cfg.cpu().numpy(), lp.cpu().numpy())
    assert n >= 30


def test_direct_zero_diagonal_weight():
    """b_diag = 0 excludes diagonal digits (s = s') from p_4: on random
    tensors no drawn digit is diagonal; on the exact beta = 0 identity, where
    only diagonal digits have nonzero marginals, no digit is left, and every
    chain reports a zero amplitude with log p = -inf and zero digits."""
    import paper_2409_05285_amd as p
    dev = _dev()
    _say("direct b_diag = 0")
    desc = p.Desc(3, 3, 2, 4)
    b = torch.zeros(1, dtype=torch.float64, device=dev)
    th = torch.tensor(synth.theta_random_unit(3, 3, 2, 2, seed=131), device=dev)
    cfg, lp, st = p.peps_direct_sample(desc, th, 64, 16, seed=61, reweight=True, b_diag=b)
    torch.cuda.synchronize()
    assert p.check(st) == 0
    c = cfg.cpu().numpy()
    assert np.all(c // 2 != c % 2)
    assert np.all(np.isfinite(lp.cpu().numpy()))
    th0 = torch.tensor(synth.theta_identity(3, 3, 2, 2, noise=0.0, seed=0), device=dev)
    cfg, lp, st = p.peps_direct_sample(desc, th0, 16, 16, seed=61, reweight=True, b_diag=b)
    torch.cuda.synchronize()
    assert st.item() == -6
    assert np.all(lp.cpu().numpy() == -np.inf)
    assert np.all(cfg.cpu().numpy() == 0)
