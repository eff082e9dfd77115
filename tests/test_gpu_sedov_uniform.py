"""The uniform-grid blast (the paper's 3D Sedov runs, and its MHD blast series) on the GPU.

* Parity: the first steps at 32^3, hydro and MHD (uniform field B = (0.01, 0, 0)), FP64
  bitwise against the oracle.
* Accuracy: at 128^3 the shock radius follows the similarity law R = xi0 (E t^2/rho)^(1/5)
  to within one cell at every sampled time, and the fitted exponent is 2/5 to 0.02.
"""
import numpy as np
import pytest

from paper_0910_5547_amd import workloads as W
from tests.gpu_util import active_all, log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from oracle import oracle as O
    from paper_0910_5547_amd import amr as A
    A.lib()
    return torch, A, O


@pytest.mark.parametrize("nvar,B0", [(5, 0.0), (8, 0.01)])
def test_blast_first_steps_match_oracle(env, nvar, B0):
    torch, A, O = env
    log(f"case sedov uniform 32 nvar={nvar}")
    ps, U, sol = W.sedov_uniform(32, t0=0.01, nvar=nvar, B0=B0)
    T = A.Table(ps, precision=0)
    Ud = T.upload(U)
    o = O.Oracle(ps)
    Uo = U.copy()
    for s in range(4):
        dt = T.cfl_dt(Ud, 0.8)
        assert dt == o.cfl_dt(Uo, 0.8), s
        T.step(Ud)
        assert o.rk2_step(Uo, dt) == 0
    assert T.status() == A.AMR_OK
    g = active_all(ps, Ud.cpu().numpy())
    T.close()
    assert np.array_equal(g, active_all(ps, Uo))


@pytest.mark.parametrize("prec", [0, 1])
def test_shock_radius_follows_similarity_law(env, prec):
    torch, A, O = env
    log(f"case sedov uniform 128 prec={prec}")
    N = 128
    ps, U, sol = W.sedov_uniform(N, t0=0.01)
    T = A.Table(ps, precision=prec)
    Ud = T.upload(U)
    t, times, radii = 0.01, [], []
    for t_next in (0.0125, 0.015, 0.0175, 0.02):
        while t < t_next - 1e-15:
            dt = min(T.cfl_dt(Ud, 0.8), t_next - t)
            T.step(Ud, dt=dt)
            t += dt
        R = W.shock_radius(ps, Ud.cpu().numpy())
        times.append(t)
        radii.append(R)
        log(f"t={t:.4f} R={R:.4f} exact={sol.radius(1.0, t):.4f} ({(R - sol.radius(1.0, t)) * N:+.2f} cells)")
        assert abs(R - sol.radius(1.0, t)) <= 1.0 / N
    assert T.status() == A.AMR_OK
    T.close()
    slope = np.polyfit(np.log(times), np.log(radii), 1)[0]
    log(f"fitted exponent {slope:.4f}")
    assert abs(slope - 0.4) <= 0.02
