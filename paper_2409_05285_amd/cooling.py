"""Cooling loop over the library calls, with one log record per SR step.

One step (Method section, Eqs. 5-7): `sweeps_per_step` Metropolis sweeps of
every chain with a measurement after each (one `peps_sample_sweep` call),
then the SR solve on all samples with theta updated in place
(`sr_cg_solve`).  After n steps the state approximates exp(-n tau calH)|I>,
whose energy E = Ebar / 2 belongs to inverse temperature beta_phys =
4 n tau.  With alpha = 1 (Appendix A) the samples are drawn from |rho| and
every average, the SR metric included, is weighted by |rho| (Eq. A1).

The state of a run is (theta, configurations, next global sweep index): a
run resumed from a saved state with `gsweep0` and `step0` continues the
same chain of states bit for bit.

Host orchestration only: every contraction, factorisation and reduction
runs in the library's kernels; the host reads back the per-sample
log-amplitudes and local energies for the log record (and, for alpha = 1,
forms the weights |rho| / max |rho| from the log-amplitudes).
"""
from __future__ import annotations

import json
import time

import numpy as np
import torch

from . import api


def _mean_and_stderr(values, w):
    """Weighted mean over all samples of [S, n] values and the standard
    error of the per-chain weighted means."""
    m = float((w * values).sum() / w.sum())
    chain = (w * values).sum(axis=0) / w.sum(axis=0)
    se = float(chain.std(ddof=1) / np.sqrt(chain.size)) if chain.size > 1 else 0.0
    return m, se


def cool(desc: api.Desc, theta, configs, n_steps, sweeps_per_step, tau, eps, seed, cg_iters=200, rtol=1e-10,
         step0=0, gsweep0=0, log=None, observables=False, su_steps=0):
    """Run n_steps SR steps; theta (float64 [N_p], device) and configs (uint8
    [n_chains, N], device) are updated in place.  `log`: a text stream that
    receives one JSON line per step.  Returns the list of records:
      step, beta_phys (of the samples of this step, 4 tau step), E_per_site
      and its standard error from the chain means, accepted moves per chain
      and sweep (horizontal exchange, site move, vertical exchange), CG
      iterations and relative residual |r| / |b|, |dtheta|, samples/s of the
      step (wall clock), and gsweep, the global sweep index the next step
      starts from.
    With observables=True each record also holds, from the same samples
    and weights (Benchmark section), with standard errors: <M_z^2>/N and the
    susceptibility beta_phys <M_z^2>/N, the particle number and double
    occupancy per site (Hubbard), and the next-nearest-neighbour spin
    correlation F (one more evaluation of the samples, before the update).
    su_steps > 0: first that many simple-update steps of tau from unit bond
    weights (the high-temperature alternative to SR; spin-1/2 Heisenberg with
    J2 = 0), the weights absorbed into theta, then n_steps SR steps numbered
    from step0 + su_steps (so beta_phys keeps counting 4 tau per step)."""
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
    records = []
    for step in range(step0, step0 + n_steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        n_accept.zero_()
        api.peps_sample_sweep(desc, theta, configs, seed, gsweep, S, n_accept=n_accept, status=status, out=out)
        gsweep += S
        la = out["log_abs"].cpu().numpy()
        weights = None
        if desc.alpha == 1:
            w = np.exp(la - la.max())
            weights = torch.tensor(w.reshape(S * n), device=dev)
        obs = None
        if observables:
            samples = out["configs"].view(S * n, N)
            vals = api.peps_observables_batch(desc, samples).cpu().numpy().reshape(S, n, -1)
            _, f_loc = api.nnn_spin_correlation(desc, theta, samples)
            obs = (vals, f_loc.cpu().numpy().reshape(S, n))
        dtheta, _, stats, _ = api.sr_cg_solve(desc, out["configs"].view(S * n, N), out["O"].view(S * n, nnz),
                                              out["e_loc"].view(S * n), tau, eps, cg_iters, rtol, weights=weights,
                                              want_g=False, theta=theta, status=status)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        api.check(status, "cool")
        e = out["e_loc"].cpu().numpy() / (2 * N)
        w = np.exp(la - la.max()) if desc.alpha == 1 else np.ones_like(e)
        chain = (w * e).sum(axis=0) / w.sum(axis=0)
        st = stats.cpu().numpy()
        acc = n_accept.cpu().numpy().sum(axis=0) / float(n * S)
        rec = {"step": step, "beta_phys": 4.0 * tau * step, "E_per_site": float(st[0]) / (2 * N),
               "E_stderr": float(chain.std(ddof=1) / np.sqrt(n)) if n > 1 else 0.0,
               "accepted_per_sweep": {"h": float(acc[0]), "site": float(acc[1]), "v": float(acc[2])},
               "cg_iters": int(st[2]), "cg_rel_residual": float(st[1] / st[3]) if st[3] > 0 else 0.0,
               "dtheta_norm": float(np.linalg.norm(dtheta.cpu().numpy())), "samples_per_s": n * S / wall,
               "gsweep": gsweep}
        if obs is not None:
            vals, f_loc = obs
            M = 2 * (desc.L1 - 1) * (desc.L2 - 1)
            for k, name in ((1, "mz2_per_site"), (2, "n_per_site"), (3, "docc_per_site")):
                m, se = _mean_and_stderr(vals[:, :, k] / N, w)
                rec[name], rec[name + "_stderr"] = m, se
            rec["chi"] = rec["beta_phys"] * rec["mz2_per_site"]
            rec["F"], rec["F_stderr"] = _mean_and_stderr(f_loc / (2.0 * M), w)
        records.append(rec)
        if log is not None:
            log.write(json.dumps(rec) + "\n")
            log.flush()
    return records
