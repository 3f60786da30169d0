"""One SR step (sweep with fused measurement, CG solve, parameter update)
captured once in a HIP graph and replayed: every replay must reproduce the
eager step bit for bit, including fresh random numbers per replay through
the device sweep counter.  Eager work and synchronisations run between the
replays, and every replay is checked, not only the last.
"""
import sys

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    return torch.device("cuda:0")


class _State:
    def __init__(self, p, desc, th, cfg, dev):
        n, nnz = cfg.shape[0], p.peps_orow_count(desc)
        self.theta = torch.tensor(th, device=dev)
        self.configs = torch.tensor(cfg, device=dev)
        self.ctr = torch.zeros(1, dtype=torch.int64, device=dev)
        self.n_accept = torch.zeros((n, 3), dtype=torch.int32, device=dev)
        self.status = p.new_status(dev)
        # caller-owned workspaces: a captured call must not see them reallocated
        self.ws = torch.empty(p.workspace_bytes(desc, n, "sweep"), dtype=torch.uint8, device=dev)
        self.ws_sr = torch.empty(p.workspace_bytes(desc, n, "sr"), dtype=torch.uint8, device=dev)
        self.out = {"log_abs": torch.empty((1, n), dtype=torch.float64, device=dev),
                    "sign": torch.empty((1, n), dtype=torch.int8, device=dev),
                    "e_loc": torch.empty((1, n), dtype=torch.float64, device=dev),
                    "O": torch.empty((1, n, nnz), dtype=torch.float64, device=dev)}

    def snapshot(self):
        return (self.configs.cpu().numpy().copy(), self.theta.cpu().numpy().copy(),
                self.out["e_loc"].cpu().numpy().copy(), self.n_accept.cpu().numpy().copy(),
                int(self.ctr.item()))


def _step(p, desc, s, seed, tau, eps):
    p.peps_sample_sweep(desc, s.theta, s.configs, seed, 0, 1, n_accept=s.n_accept, status=s.status, out=s.out,
                        sweep_counter=s.ctr, ws=s.ws)
    p.sr_cg_solve(desc, s.configs, s.out["O"][0], s.out["e_loc"][0], tau, eps, 30, 0.0, want_g=False,
                  theta=s.theta, status=s.status, ws=s.ws_sr)


@pytest.mark.parametrize("mixed", [False, True])
def test_graph_replay_matches_eager(mixed):
    dev = _dev()
    import paper_2409_05285_amd as p
    print("[case] graph replay", "mixed" if mixed else "fp64", flush=True)
    sys.stdout.flush()
    L1, L2, D, chi, n = 4, 4, 2, 4, 16
    desc = p.Desc(L1, L2, D, chi, precision=p.PREC_MIXED if mixed else p.PREC_FP64)
    th = synth.theta_identity(L1, L2, D, 2, noise=0.05, seed=31)
    cfg = synth.configs_diagonal(n, L1 * L2, 2, seed=32)
    seed, tau, eps, steps = 555, 0.01, 1e-3, 4

    eager = _State(p, desc, th, cfg, dev)
    ref = []
    for _ in range(steps):
        _step(p, desc, eager, seed, tau, eps)
        torch.cuda.synchronize()
        assert p.check(eager.status) in (0, 1)   # 1: CG at its fixed iteration count
        ref.append(eager.snapshot())
    # the counter really advanced the random numbers: consecutive sweeps differ
    assert ref[-1][4] == steps

    g_state = _State(p, desc, th, cfg, dev)
    graph = torch.cuda.CUDAGraph()
    torch.cuda.synchronize()
    with torch.cuda.graph(graph):
        _step(p, desc, g_state, seed, tau, eps)
    torch.cuda.synchronize()
    # capture records only: the state is still the initial one
    assert np.array_equal(g_state.configs.cpu().numpy(), cfg)
    side = torch.tensor(th, device=dev)
    for k in range(steps):
        graph.replay()
        # unrelated eager work between replays
        side.mul_(1.0000001).add_(1e-9)
        p.peps_eval_batch(desc, side, g_state.configs.clone())
        torch.cuda.synchronize()
        assert p.check(g_state.status) in (0, 1)
        got = g_state.snapshot()
        assert np.array_equal(got[0], ref[k][0]), k
        assert np.array_equal(got[1], ref[k][1]), k
        assert np.array_equal(got[2], ref[k][2]), k
        assert np.array_equal(got[3], ref[k][3]), k
        assert got[4] == ref[k][4], k
