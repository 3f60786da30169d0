"""Cooling loop (Method section and Appendix A): start from the beta = 0
identity state with small perturbations, then repeat
    sample -> (E_loc, O) -> SR solve -> theta += dtheta.
One SR step approximates |rho> <- exp(-tau calH)|rho> (Eq. (5) and the text
before it).  After n steps |rho> ~ exp(-n tau calH)|I> = |rho_beta> with
beta / 2 = n tau, and the estimated energy E = Ebar / 2 (Eq. (in_en)) belongs
to inverse temperature 2 beta = 4 n tau (reading of the bookkeeping).
"""
from __future__ import annotations

import numpy as np

from . import measure, sampler, sr


def cool(lat, theta0, configs0, chi, seed, n_steps, sweeps_per_step, tau, eps,
         max_iter=200, rtol=1e-10, alpha=2, log=None, gsweep0=0, step0=0):
    """n_steps SR steps from (theta0, configs0).  The Metropolis uniforms are
    positional in (chain, global sweep, slot), so a run resumed from saved
    (theta, configs, gsweep, step) with gsweep0 and step0 continues the same
    chain of states; every history record carries the global sweep index
    the next step would start from."""
    theta = np.array(theta0, dtype=np.float64, copy=True)
    configs = np.array(configs0, dtype=np.int64, copy=True)
    n_chains = configs.shape[0]
    gsweep = gsweep0
    history = []
    for step in range(step0, step0 + n_steps):
        samples, e_list, o_list = [], [], []
        for k in range(sweeps_per_step):
            for ch in range(n_chains):
                res = sampler.sweep(lat, theta, configs[ch], chi, seed, ch, gsweep, alpha=alpha)
                configs[ch] = res["S"]
                ev = measure.evaluate(lat, theta, res["S"], chi)
                samples.append(res["S"].copy())
                e_list.append(ev["e_loc"])
                o_list.append(ev["O"])
            gsweep += 1
        sol = sr.sr_solve(lat, np.array(samples), np.array(o_list), np.array(e_list),
                          tau, eps, max_iter, rtol)
        theta = theta + sol["dtheta"]
        e = np.array(e_list)
        rec = {"step": step, "beta_phys": 4.0 * tau * step, "E_per_site": sol["ebar"] / (2 * lat.N),
               "sigma": float(e.std(ddof=1) / np.sqrt(len(e)) / (2 * lat.N)) if len(e) > 1 else 0.0,
               "cg_iters": sol["iters"], "gsweep": gsweep}
        history.append(rec)
        if log is not None:
            log(rec)
    return theta, configs, history
