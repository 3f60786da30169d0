"""Next-nearest-neighbour spin correlation on the Hubbard lattice (Benchmark
section: F = sum_<<ij>> <S_i.S_j> / M, M the number of such pairs).

The device evaluates it as the local energy of J2 sum_<<ij>> S_i.S_j, a term
the Hubbard descriptor carries next to t, U and mu (S^+ = c^dag_up c_dn, no
Jordan-Wigner sign on the exchange).

* Parity: log|psi|, sign, E_loc and O of the Hubbard model with J2 != 0
  against the oracle on sector-consistent configurations (FP64 1e-10 / 1e-9,
  mixed 1e-4), exact and truncating boundary dimensions.
* Estimator: on 2x2 (chi exact) every one of the 16^4 configurations is
  evaluated on the device and weighted by |rho|^2; the resulting F equals
  Tr(rho rho^T A + rho^T rho A) / (2 M Tr(rho rho^T)) with rho the oracle's
  dense density matrix and A = sum_<<ij>> S_i.S_j built from fermion mode
  operators.
"""
import sys

import numpy as np
import pytest

import synth
from oracle import hamiltonian, measure, network
from oracle.lattice import MODEL_HUBBARD, Lattice

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    return torch.device("cuda:0")


def _say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("L1,L2,D,chi,mixed", [(4, 4, 2, 4, False), (4, 5, 2, 3, False), (4, 4, 2, 4, True)])
def test_hubbard_nnn_exchange_matches_oracle(L1, L2, D, chi, mixed):
    dev = _dev()
    import paper_2409_05285_amd as p
    _say("hubbard + J2 eval", L1, L2, D, chi, "mixed" if mixed else "fp64")
    J2 = 0.6
    lat = Lattice(L1, L2, D=D, chi=chi, d=4, model=MODEL_HUBBARD, t=1.0, U=8.0, mu=4.0, J2=J2)
    desc = p.Desc(L1, L2, D, chi, d=4, model=p.MODEL_HUBBARD, t=1.0, U=8.0, mu=4.0, J2=J2,
                  precision=p.PREC_MIXED if mixed else p.PREC_FP64)
    th = synth.theta_random_unit(L1, L2, D, 4, seed=81)
    cfg = synth.configs_sector(6, lat.N, 4, seed=82)
    theta_d = torch.tensor(th, device=dev)
    cfg_d = torch.tensor(cfg, device=dev)
    la, sg, el, st = p.peps_eval_batch(desc, theta_d, cfg_d)
    O, _, st2 = p.peps_grad_batch(desc, theta_d, cfg_d)
    torch.cuda.synchronize()
    assert p.check(st) == 0 and p.check(st2) == 0
    ref = measure.evaluate_batch(lat, th, cfg, chi)
    # the exchange terms are present in these samples
    n_exch = sum(1 for S in cfg for _, _, info in hamiltonian.terms(lat, S)[1] if info[2] == "d")
    assert n_exch > 0
    la, sg, el, O = (x.cpu().numpy() for x in (la, sg, el, O))
    tol = 1e-4 if mixed else 1e-10
    assert np.all(np.abs(la - ref["log_abs"]) <= tol * np.maximum(1.0, np.abs(ref["log_abs"])))
    assert np.array_equal(sg, ref["sign"])
    emag = max(np.abs(ref["e_loc"]).mean(), 1e-300)
    assert np.all(np.abs(el - ref["e_loc"]) <= tol * np.maximum(np.abs(ref["e_loc"]), emag)), (el, ref["e_loc"])
    otol = 1e-4 * np.maximum(1.0, np.abs(ref["O"]).max(axis=1, keepdims=True)) if mixed else \
        1e-9 * np.maximum(1.0, np.abs(ref["O"]))
    assert np.all(np.abs(O - ref["O"]) <= otol)


def test_nnn_spin_correlation_by_enumeration():
    dev = _dev()
    import paper_2409_05285_amd as p
    _say("F by enumeration, 2x2 Hubbard D=2")
    lat = Lattice(2, 2, D=2, chi=4, d=4, model=MODEL_HUBBARD, t=0.0, U=0.0, mu=0.0, J2=1.0)
    desc = p.Desc(2, 2, 2, 4, d=4, model=p.MODEL_HUBBARD, t=1.0, U=8.0, mu=4.0)
    th = synth.theta_random_unit(2, 2, 2, 4, seed=71)
    theta_d = torch.tensor(th, device=dev)
    allc = np.ascontiguousarray(np.array(np.unravel_index(np.arange(16 ** 4), (16,) * 4)).T.astype(np.uint8))
    cfg_d = torch.tensor(allc, device=dev)
    la, _, _, st = p.peps_eval_batch(desc, theta_d, cfg_d)
    torch.cuda.synchronize()
    assert p.check(st) == 0
    w = torch.exp(2.0 * (la - la.max()))
    F, _, e = p.nnn_spin_correlation(desc, theta_d, cfg_d, weights=w.contiguous())
    rho = network.density_matrix(lat, th)
    A = hamiltonian.dense_H(lat)
    M = 2
    F_ref = float(np.trace(rho @ rho.T @ A + rho.T @ rho @ A) / (2 * M * np.trace(rho @ rho.T)))
    print("[F] device %.15f oracle %.15f" % (F, F_ref), flush=True)
    assert abs(F - F_ref) <= 1e-10 * max(1.0, abs(F_ref))
    # the unweighted estimator on the diagonal configurations of |I> is 0
    diag = torch.tensor([[4 * s + s for s in sv] for sv in np.ndindex(4, 4, 4, 4)], dtype=torch.uint8, device=dev)
    th_id = torch.tensor(synth.theta_identity(2, 2, 2, 4), device=dev)
    F0, _, _ = p.nnn_spin_correlation(desc, th_id, diag)
    assert abs(F0) <= 1e-14
