"""Batched uneven instances (sch_batch_*) versus the oracle's bootstrap
cycle run for each instance alone, with the instance's own seed.

Same bars as the single-filter bootstrap parity: states within relative L2
1e-10, log-weights and ESS to 1e-9, identical resampling decisions."""
import sys

import numpy as np
import pytest

import oracle as O
import pairing as PR
from paper_2402_06927_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def sch():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2402_06927_amd import sch as S

    S.lib()
    return S


def T(a, dtype=torch.float64):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def N(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def _instance_workload(base, inst):
    return base.scaled(nx=inst.nx, n_particles=inst.n_particles, seed=inst.seed)


def _setup(sch, base, insts, n_cycles, threads=None, checked=None):
    """GPU instances plus, for the checked ones, the oracle's inputs."""
    gi, ref = [], {}
    for k, ins in enumerate(insts):
        if k % 8 == 0:
            _say("  set-up of instance", k, "of", len(insts))
        wl = _instance_workload(base, ins)
        xi = T(W.mode_table(wl.L, wl.nx, wl.n_modes, wl.mode_amp))
        if checked is None or k in checked:
            u, m, _, _ = PR.prior(wl, ins.n_particles)
            ys = PR.oracle_observations(wl, n_cycles)
            ref[k] = dict(wl=wl, m=m.copy(), u=u.copy(), lw=np.zeros(ins.n_particles), ys=ys)
            mt, ut = T(m), T(u)
        else:
            u = W.initial_velocity(wl, ins.n_particles, wl.seed)
            ut = T(u)
            mt = torch.empty_like(ut)
            gm = PR.gpu_model(wl)
            sch.sch_init_momentum(gm, ut, mt)
            x = W.node_positions(wl.L, wl.nx)
            y0 = np.interp(np.arange(wl.n_obs) * wl.L / wl.n_obs, x, u.mean(axis=0))
            ys = np.tile(y0, (n_cycles, 1))
        gi.append(sch.Instance(xi=xi, m=mt, u=ut,
                               logw=torch.zeros(ins.n_particles, dtype=torch.float64,
                                                device="cuda"),
                               y=T(ys), sigma=T(np.full(wl.n_obs, wl.sigma_obs)), seed=ins.seed,
                               threads=(threads[k] if threads else 0)))
    b = sch.Batch(base.L, base.alpha, base.mu, base.dt, base.n_modes, base.n_steps, base.n_obs,
                  base.ess_frac, gi, base.picard_tol, base.picard_max)
    return b, gi, ref


def _oracle_cycle(r, c):
    wl = r["wl"]
    om = PR.oracle_model(wl)
    rc, r["m"], r["u"], r["lw"], st = O.bootstrap_cycle(
        om, r["ys"][c], np.full(wl.n_obs, wl.sigma_obs), wl.seed, c, r["m"], r["u"], r["lw"],
        wl.n_steps, wl.ess_frac)
    assert rc == 0
    return st


def _compare(b, gi, ref, c, res_prev):
    out = b.read()
    for k, r in ref.items():
        st = _oracle_cycle(r, c)
        assert out["status"][k] == 0
        assert abs(out["ess"][k] - st.ess) <= 1e-9 * st.ess, (k, c)
        assert out["resampled"][k] - res_prev[k] == st.resampled, (k, c)
        assert PR.rel_l2(N(gi[k].m), r["m"]) < PR.REL_TOL, (k, c)
        assert PR.rel_l2(N(gi[k].u), r["u"]) < PR.REL_TOL, (k, c)
        np.testing.assert_allclose(N(gi[k].logw), r["lw"], rtol=1e-9, atol=1e-9)
    return out["resampled"]


@pytest.mark.parametrize("use_graph", [False, True])
def test_batch_parity_small(sch, use_graph):
    """Eight instances with ragged grids (nx in [64, 1200]) and ensembles in
    [4, 48], bootstrap physics of the Nx = 256 workload, three cycles; two
    instances force their threads per particle."""
    base = W.BOOTSTRAP_256
    insts = W.uneven_instances(8, nx_range=(64, 1200), np_range=(4, 48))
    threads = [0] * len(insts)
    # one instance on 64 threads (up to 16 nodes each), one on 256 threads
    k64 = next(k for k, i in enumerate(insts) if 128 <= i.nx <= 1024)
    threads[k64] = 64
    k256 = next((k for k, i in enumerate(insts) if i.nx >= 256 and k != k64), None)
    if k256 is not None:
        threads[k256] = 256
    _say("batch small", [(i.nx, i.n_particles) for i in insts], threads, use_graph)
    b, gi, ref = _setup(sch, base, insts, 3, threads=threads)
    res = [0] * len(insts)
    for c in range(3):
        b.run(c, 1, use_graph=use_graph)
        res = _compare(b, gi, ref, c, res)
    assert sum(res) >= 1
    b.close()


def test_batch_graph_replays_match_direct_launches(sch):
    base = W.BOOTSTRAP_256.scaled(n_steps=8)
    insts = W.uneven_instances(5, seed=77, nx_range=(64, 700), np_range=(8, 40))
    runs = []
    for use_graph in (True, False):
        b, gi, _ = _setup(sch, base, insts, 4, checked=set())
        b.run(0, 4, use_graph=use_graph)
        out = b.read()
        runs.append(([N(g.m) for g in gi], [N(g.logw) for g in gi], out))
        b.close()
    for a, c in zip(runs[0][0], runs[1][0]):
        np.testing.assert_array_equal(a, c)
    for a, c in zip(runs[0][1], runs[1][1]):
        np.testing.assert_array_equal(a, c)
    assert runs[0][2]["resampled"] == runs[1][2]["resampled"]
    assert runs[0][2]["picard_iters"] == runs[1][2]["picard_iters"]


def test_batch_rejects_bad_instances(sch):
    """Shape and argument errors are reported before any device work."""
    base = W.BOOTSTRAP_256.scaled(n_steps=2)
    insts = W.uneven_instances(2, seed=5, nx_range=(64, 128), np_range=(4, 8))

    def make(threads=0, y=True):
        gi = []
        for ins in insts:
            z = torch.zeros((ins.n_particles, ins.nx), dtype=torch.float64, device="cuda")
            gi.append(sch.Instance(
                xi=torch.zeros((base.n_modes, ins.nx), dtype=torch.float64, device="cuda"),
                m=z, u=z.clone(),
                logw=torch.zeros(ins.n_particles, dtype=torch.float64, device="cuda"),
                y=torch.zeros((1, base.n_obs), dtype=torch.float64, device="cuda") if y else None,
                sigma=torch.ones(base.n_obs, dtype=torch.float64, device="cuda"),
                seed=ins.seed, threads=threads))
        return gi

    def batch(gi):
        return sch.Batch(base.L, base.alpha, base.mu, base.dt, base.n_modes, base.n_steps,
                         base.n_obs, base.ess_frac, gi)

    with pytest.raises(sch.SchError, match="NULL"):
        batch(make(y=False))
    with pytest.raises(sch.SchError, match="no tile"):
        batch(make(threads=256))  # more threads than nodes
    with pytest.raises(sch.SchError, match="no tile"):
        batch(make(threads=96))   # not a power of two


def test_batch_full_size_sampled(sch):
    """The 64-instance workload at full size (nx log-uniform in [512, 8192],
    ensembles log-uniform in [64, 2048]); the three smallest instances are
    checked against the oracle for one cycle."""
    base = W.BOOTSTRAP_256
    insts = W.uneven_instances(64)
    sizes = [i.nx * i.n_particles for i in insts]
    checked = set(int(k) for k in np.argsort(sizes)[:3])
    _say("batch full", sum(sizes), "node-states; checked", checked)
    b, gi, ref = _setup(sch, base, insts, 1, checked=checked)
    b.run(0, 1, use_graph=False)
    _compare(b, gi, ref, 0, [0] * len(insts))
    out = b.read()
    assert all(s == 0 for s in out["status"])
    b.close()
