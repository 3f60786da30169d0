"""Cooling loop over the library calls, with one log record per SR step.

One step (Method section, Eqs. 5-7): `sweeps_per_step` Metropolis sweeps of
every chain with a measurement after each (one `peps_sample_sweep` call),
then the SR solve on all samples with theta updated in place
(`sr_cg_solve`).  After n steps the state approximates exp(-n tau calH)|I>,
whose energy E = Ebar / 2 belongs to inverse temperature beta_phys =
4 n tau.  With alpha = 1 (Appendix A) the samples are drawn from |rho| and
every average, the SR metric included, is weighted by |rho| (Eq. A1); the
weights are formed on the device from the log-amplitudes.  The paper samples
this way at high temperature only and switches to |rho|^2 sampling near
beta = 0.3 (Benchmark section, Heisenberg paragraph): `alpha_switch_beta`
sets that temperature.

The state of a run is (theta, configurations, next global sweep index): a
run resumed from a saved state with `gsweep0` and `step0` continues the
same chain of states bit for bit.

Host orchestration only: every contraction, factorisation, weight and
reduction runs in the library's kernels (the means and standard errors of
the log record by peps_sample_stats); the host reads back those few scalars.
"""
from __future__ import annotations

import dataclasses
import json
import time

import torch

from . import api


def cool(desc: api.Desc, theta, configs, n_steps, sweeps_per_step, tau, eps, seed, cg_iters=200, rtol=1e-10,
         step0=0, gsweep0=0, log=None, observables=False, su_steps=0, alpha_switch_beta=None, sampler="metropolis",
         chi_dl=None, reweight=True, b_diag0=1.0):
    """Run n_steps SR steps; theta (float64 [N_p], device) and configs (uint8
    [n_chains, N], device) are updated in place.  `log`: a text stream that
    receives one JSON line per step.  Returns the list of records:
      step, beta_phys (of the samples of this step, 4 tau step), alpha (the
      sampling exponent of the step), E_per_site and its standard error
      from the chain means, accepted moves per chain and sweep (horizontal
      exchange, site move, vertical exchange), CG iterations, relative
      residual |r| / |b| and whether the residual bar was met, |dtheta|,
      samples/s of the step (wall clock), and gsweep, the global sweep index
      the next step starts from.
    alpha_switch_beta: with desc.alpha = 1, the steps whose beta_phys is at
    or above this value sample |rho|^2 instead (alpha = 2, uniform weights).
    With observables=True each record also holds, from the same samples
    and weights (Benchmark section), with standard errors: <M_z^2>/N and the
    susceptibility beta_phys <M_z^2>/N, the particle number and double
    occupancy per site (Hubbard), and the next-nearest-neighbour spin
    correlation F (one more evaluation of the samples, before the update).
    su_steps > 0: first that many simple-update steps of tau from unit bond
    weights (the high-temperature alternative to SR; spin-1/2 Heisenberg with
    J2 = 0), the weights absorbed into theta, then n_steps SR steps numbered
    from step0 + su_steps (so beta_phys keeps counting 4 tau per step).
    sampler="direct": instead of Metropolis sweeps, every step draws
    sweeps_per_step independent configurations per chain by direct sampling
    (Appendix A; p_4 with the dynamic diagonal weight when reweight, else
    p_2; double-layer boundary dimension chi_dl, default chi^2), evaluates
    them, and weights every average and the SR metric by r = |rho|^2 / p
    (Eq. A7).  The diagonal weight starts at b_diag0 and is updated on the
    device after the last draw of each step; records then also hold
    "b_diag" and "sampler", and accepted_per_sweep is None.  `configs`
    receives the last draw."""
    n = configs.shape[0]
    S = int(sweeps_per_step)
    N = desc.N
    nnz = api.peps_orow_count(desc)
    dev = theta.device
    status = api.new_status(dev)
    out = {
        "log_abs": torch.empty((S, n), dtype=torch.float64, device=dev),
        "sign": torch.empty((S, n), dtype=torch.int8, device=dev),
        "e_loc": torch.empty((S, n), dtype=torch.float64, device=dev),
        "O": torch.empty((S, n, nnz), dtype=torch.float64, device=dev),
        "configs": torch.empty((S, n, N), dtype=torch.uint8, device=dev),
    }
    n_accept = torch.zeros((n, 3), dtype=torch.int32, device=dev)
    gsweep = int(gsweep0)
    if su_steps > 0:
        lam = torch.ones((api.su_bond_count(desc), desc.D), dtype=torch.float64, device=dev)
        api.peps_simple_update(desc, theta, lam, tau, su_steps, status=status)
        theta.copy_(api.peps_su_absorb(desc, theta, lam))
        torch.cuda.synchronize()
        api.check(status, "simple update")
        step0 = step0 + su_steps
    direct = sampler == "direct"
    if sampler not in ("metropolis", "direct"):
        raise ValueError("sampler must be 'metropolis' or 'direct'")
    if direct:
        chi_dl = desc.chi * desc.chi if chi_dl is None else int(chi_dl)
        b_diag = torch.tensor([float(b_diag0)], dtype=torch.float64, device=dev)
        log_p = torch.empty(S * n, dtype=torch.float64, device=dev)
        dws = torch.empty(api.peps_direct_workspace_bytes(desc, n, chi_dl), dtype=torch.uint8, device=dev)
    records = []
    for step in range(step0, step0 + n_steps):
        beta_phys = 4.0 * tau * step
        d = desc
        if desc.alpha == 1 and alpha_switch_beta is not None and beta_phys >= alpha_switch_beta:
            d = dataclasses.replace(desc, alpha=2)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        samples = out["configs"].view(S * n, N)
        w = None
        if direct:
            for k in range(S):
                sl = slice(k * n, (k + 1) * n)
                # the draws of one step share theta: the double layer is built by the first
                api.peps_direct_sample(d, theta, n, chi_dl, seed, draw=gsweep + k, reweight=reweight, b_diag=b_diag,
                                       update_b=reweight and k == S - 1, reuse_double_layer=k > 0, status=status,
                                       out=(samples[sl], log_p[sl]), ws=dws)
            configs.copy_(samples[(S - 1) * n:])
            la, _, e, _ = api.peps_eval_batch(d, theta, samples, status=status)
            O, _, _ = api.peps_grad_batch(d, theta, samples, status=status)
            w = api.peps_importance_weights(la, log_p)
        else:
            n_accept.zero_()
            api.peps_sample_sweep(d, theta, configs, seed, gsweep, S, n_accept=n_accept, status=status, out=out)
            la = out["log_abs"].view(S * n)
            e = out["e_loc"].view(S * n)
            O = out["O"].view(S * n, nnz)
        gsweep += S
        wa = {"weights": w} if direct else {"log_abs": la}
        est = api.peps_sample_stats(d, e, n, **wa)
        obs = None
        if observables:
            vals = api.peps_observables_batch(d, samples)
            ost = api.peps_sample_stats(d, vals, n, **wa)
            f_mean, f_se, _ = api.nnn_spin_correlation(d, theta, samples, n_chains=n, **wa)
            obs = (ost, f_mean, f_se)
        dtheta, _, stats, _ = api.sr_cg_solve(d, samples, O, e, tau, eps, cg_iters, rtol, want_g=False, theta=theta,
                                              status=status, **wa)
        dnorm = torch.linalg.vector_norm(dtheta)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        api.check(status, "cool")
        est = est.cpu().tolist()
        st = stats.cpu().tolist()
        acc = None if direct else (n_accept.sum(dim=0).to(torch.float64) / float(n * S)).cpu().tolist()
        rec = {"step": step, "beta_phys": beta_phys, "alpha": d.alpha,
               "E_per_site": est[0][0] / (2 * N), "E_stderr": est[0][1] / (2 * N),
               "accepted_per_sweep": None if acc is None else {"h": acc[0], "site": acc[1], "v": acc[2]},
               "cg_iters": int(st[2]), "cg_rel_residual": st[1] / st[3] if st[3] > 0 else 0.0,
               "cg_converged": st[4] == 0.0,
               "dtheta_norm": float(dnorm), "samples_per_s": n * S / wall, "gsweep": gsweep}
        if direct:
            rec["sampler"], rec["b_diag"] = "direct", float(b_diag.item())
        if obs is not None:
            ost, f_mean, f_se = obs
            ost = ost.cpu().tolist()
            for q, name in ((1, "mz2_per_site"), (2, "n_per_site"), (3, "docc_per_site")):
                rec[name], rec[name + "_stderr"] = ost[q][0] / N, ost[q][1] / N
            rec["chi"] = beta_phys * rec["mz2_per_site"]
            rec["F"], rec["F_stderr"] = f_mean, f_se
        records.append(rec)
        if log is not None:
            log.write(json.dumps(rec) + "\n")
            log.flush()
    return records
