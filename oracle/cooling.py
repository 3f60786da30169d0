"""Cooling loop (Method section and Appendix A): start from the beta = 0
identity state with small perturbations, then repeat
    sample -> (E_loc, O) -> SR solve -> theta += dtheta.
One SR step approximates |rho> <- exp(-tau calH)|rho> (Eq. (5) and the text
before it).  After n steps |rho> ~ exp(-n tau calH)|I> = |rho_beta> with
beta / 2 = n tau, and the estimated energy E = Ebar / 2 (Eq. (in_en)) belongs
to inverse temperature 2 beta = 4 n tau (reading of the bookkeeping).
With alpha = 1 the samples are drawn from |rho| (Appendix A) and every
average, the SR metric included, takes the weights |rho|^2 / |rho| = |rho|
(Eq. A1).

Test infrastructure only: nothing on the product path imports this package.
"""
from __future__ import annotations

import numpy as np

from . import measure, network, sampler, sr


def cool(lat, theta0, configs0, chi, seed, n_steps, sweeps_per_step, tau, eps,
         max_iter=200, rtol=1e-10, alpha=2, log=None, gsweep0=0, step0=0, exact=False):
    """n_steps SR steps from (theta0, configs0).  The Metropolis uniforms are
    positional in (chain, global sweep, slot), so a run resumed from saved
    (theta, configs, gsweep, step) with gsweep0 and step0 continues the same
    chain of states; every history record carries the global sweep index
    the next step would start from.
    exact=True (tiny lattices, chi large enough for an exact contraction):
    every step averages over all d^(2N) configurations with weights
    |rho(S)|^2 instead of sampling, so the loop follows the SR trajectory of
    exact expectations (configs, seed and sweeps_per_step are then unused)."""
    theta = np.array(theta0, dtype=np.float64, copy=True)
    configs = np.array(configs0, dtype=np.int64, copy=True)
    n_chains = configs.shape[0]
    gsweep = gsweep0
    history = []
    for step in range(step0, step0 + n_steps):
        if exact:
            samples, e_list, o_list, w = [], [], [], []
            for S in network.all_configs(lat):
                ev = measure.evaluate(lat, theta, S, chi)
                if ev["sign"] == 0:
                    continue
                samples.append(np.array(S))
                e_list.append(ev["e_loc"])
                o_list.append(ev["O"])
                w.append(ev["log_abs"])
            la = np.array(w)
            w = np.exp(2.0 * (la - la.max()))
            sol = sr.sr_solve(lat, np.array(samples), np.array(o_list), np.array(e_list), tau, eps, max_iter, rtol,
                              weights=w)
            theta = theta + sol["dtheta"]
            rec = {"step": step, "beta_phys": 4.0 * tau * step, "E_per_site": sol["ebar"] / (2 * lat.N),
                   "sigma": 0.0, "cg_iters": sol["iters"], "gsweep": gsweep}
            history.append(rec)
            if log is not None:
                log(rec)
            continue
        samples, e_list, o_list, la_list, chain_of = [], [], [], [], []
        for k in range(sweeps_per_step):
            for ch in range(n_chains):
                res = sampler.sweep(lat, theta, configs[ch], chi, seed, ch, gsweep, alpha=alpha)
                configs[ch] = res["S"]
                ev = measure.evaluate(lat, theta, res["S"], chi)
                samples.append(res["S"].copy())
                e_list.append(ev["e_loc"])
                o_list.append(ev["O"])
                la_list.append(ev["log_abs"])
                chain_of.append(ch)
            gsweep += 1
        e = np.array(e_list)
        la = np.array(la_list)
        # Eq. A1: samples drawn from |rho|^alpha estimate |rho|^2 averages
        # with weights |rho|^(2 - alpha)
        w = np.exp((2 - alpha) * (la - la.max())) if alpha != 2 else None
        sol = sr.sr_solve(lat, np.array(samples), np.array(o_list), e, tau, eps, max_iter, rtol, weights=w)
        theta = theta + sol["dtheta"]
        ww = np.ones_like(e) if w is None else w
        chain_of = np.array(chain_of)
        means = np.array([(ww[chain_of == c] * e[chain_of == c]).sum() / ww[chain_of == c].sum()
                          for c in range(n_chains)])
        rec = {"step": step, "beta_phys": 4.0 * tau * step, "E_per_site": sol["ebar"] / (2 * lat.N),
               "sigma": float(means.std(ddof=1) / np.sqrt(n_chains) / (2 * lat.N)) if n_chains > 1 else 0.0,
               "cg_iters": sol["iters"], "gsweep": gsweep}
        history.append(rec)
        if log is not None:
            log(rec)
    return theta, configs, history
