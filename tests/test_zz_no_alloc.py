"""sch_jitter_pcn_noalloc (the pCN jitter without a workspace, for callers
that cannot allocate) against sch_jitter_pcn with a caller workspace: the
same moves on the same inputs must give the same increments, potentials,
end states and acceptance counts, bit for bit (the same kernels read the same
draws).  Two calls in a row, the second smaller (and with fixed controls),
so a stale first call's draws in the library's array would show; requests
above the array's size are refused before any device work."""
import math
import sys

import numpy as np
import pytest

import oracle as O
import pairing as PR
from paper_2402_06927_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


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


def _inputs(nx, n, q, s, controls):
    wl = W.BOOTSTRAP_256.scaled(nx=nx, n_modes=q, n_steps=s, n_obs=40, sigma_obs=0.05)
    om = PR.oracle_model(wl)
    u0, m0, ut, _ = PR.prior(wl, n)
    dW = O.draw_increments(wl.seed, n, s, q, 0, O.TAG_FORECAST, 0, wl.dt)
    dL = 0.3 * math.sqrt(wl.dt) * W.random_state_noise((n, s, q), 9) if controls else None
    _, m1, u1, _, _ = O.ensemble_window(om, m0, u0, dW, dL)
    y = O.observe(ut, 40) + 0.05 * W.random_state_noise(40, 3)
    sig = np.full(40, 0.05)
    phi = O.ensemble_nll(u1, y, sig)
    if controls:
        phi = np.array([O.nudged_potential(phi[p], wl.dt, dW[p], dL[p]) for p in range(n)])
    return wl, m0, u0, dW, dL, m1, u1, y, sig, phi


def _run(sch, noalloc, wl, m0, u0, dW, dL, m1, u1, y, sig, phi, theta, n_jitter):
    gm = PR.gpu_model(wl)
    n = dW.shape[0]
    gdW, gphi, gm1, gu1 = T(dW), T(phi), T(m1), T(u1)
    acc = torch.full((n,), -1, dtype=torch.int32, device="cuda")
    args = (gm, sch.Obs(T(y), T(sig)), wl.seed, 2, 3, T(m0), T(u0), gdW, gphi, gm1, gu1,
            T([theta]), 0.95, n_jitter, acc)
    if noalloc:
        sch.sch_jitter_pcn_noalloc(*args, dLambda=None if dL is None else T(dL))
    else:
        sch.sch_jitter_pcn(*args, dLambda=None if dL is None else T(dL))
    return N(gdW), N(gphi), N(gm1), N(gu1), N(acc)


# (nx, particles, modes, steps, moves, controls): the first call at the
# headline grid and window, the second smaller everywhere
CALLS = [(4096, 64, 8, 40, 5, False), (600, 5, 4, 8, 3, True)]


def test_noalloc_jitter_equals_workspace_jitter(sch):
    cap = sch.lib().sch_jitter_pcn_noalloc_max_bytes()
    assert cap == 16 << 20
    for nx, n, q, s, nj, ctrl in CALLS:
        print("noalloc jitter", nx, n, q, s, nj, ctrl, file=sys.stderr, flush=True)
        assert 8 * (nj * n * s * q + nj * n) + 512 <= cap
        inp = _inputs(nx, n, q, s, ctrl)
        ref = _run(sch, False, *inp, 0.7, nj)
        got = _run(sch, True, *inp, 0.7, nj)
        assert 0 < ref[4].sum() < nj * n  # some moves accepted, some rejected
        for a, b in zip(got, ref):
            assert np.array_equal(a, b)


def test_noalloc_jitter_refuses_requests_above_its_array(sch):
    wl, m0, u0, dW, dL, m1, u1, y, sig, phi = _inputs(256, 3, 4, 2, False)
    # 7 moves x 1024 particles x 40 steps x 8 modes > 16 MiB of doubles:
    # shapes are checked from the arguments alone, before any device work
    n, s, q = 1024, 40, 8
    big = torch.zeros((n, s, q), dtype=torch.float64, device="cuda")
    row = torch.zeros((n, 256), dtype=torch.float64, device="cuda")
    ph = torch.zeros(n, dtype=torch.float64, device="cuda")
    gm8 = PR.gpu_model(wl.scaled(n_modes=8))
    with pytest.raises(sch.SchError) as e:
        sch.sch_jitter_pcn_noalloc(gm8, sch.Obs(T(y), T(sig)), wl.seed, 0, 0, row, row, big,
                                   ph, row.clone(), row.clone(), T([0.5]), 0.9, 7)
    assert e.value.code == sch.SCH_E_SHAPE
    assert torch.equal(big, torch.zeros_like(big))
