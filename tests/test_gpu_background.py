"""The library's coupled-quintessence background (mg_cq_background, host
FP64) against the oracle's, and a field solve that takes phi-bar(a) and lambda
from it instead of stand-ins."""
import numpy as np
import pytest
import torch

import oracle
import synthetic
from oracle import cq_background as bg
from paper_2110_00328_amd import api

pytestmark = pytest.mark.gpu
OM, H = 0.3089, 0.6774


@pytest.mark.parametrize("alpha,beta", [(0.1, -0.1), (0.1, -0.2), (0.5, -0.2), (0.0, 0.0)])
def test_background_table_matches_oracle(alpha, beta):
    info, tab = api.cq_background(alpha, beta, n_table=777)
    lam, orr, ref = bg.table(OM, H, alpha, beta, n_table=777)
    assert abs(info.lam / lam - 1.0) < 1e-10
    assert abs(info.omega_r / orr - 1.0) < 1e-13
    assert abs(info.h_today - 1.0) <= 1e-12
    for c in range(6):
        scale = np.abs(ref[:, c]).max()
        if scale == 0.0:
            assert np.all(tab[:, c] == 0.0)
        else:
            assert np.abs(tab[:, c] - ref[:, c]).max() <= 1e-9 * scale, c
    rng = np.random.default_rng(1)
    for a in np.concatenate([rng.uniform(tab[0, 0], 1.0, 20), [tab[0, 0], 1.0]]):
        assert np.allclose(api.cq_background_at(tab, a), bg.interp(tab, a), rtol=1e-13, atol=0)


def test_background_rejects_bad_input():
    with pytest.raises(api.MGError):
        api.cq_background(0.1, -0.2, omega_m=1.2)
    with pytest.raises(api.MGError):
        api.cq_background(0.1, -0.2, phi_init=0.0)
    with pytest.raises(api.MGError):
        api.cq_background(0.1, -0.2, n_table=1)
    _, tab = api.cq_background(0.1, -0.2, n_table=16)
    with pytest.raises(api.MGError):
        api.cq_background_at(tab, 1.01)
    # a coupling of the other sign drives the field through zero: reported
    with pytest.raises(api.MGError):
        api.cq_background(0.1, 5.0)


@pytest.mark.parametrize("a", [1.0, 0.5])
def test_cq_solve_with_self_consistent_background(a):
    n, box = 32, 64.0
    dev = torch.device("cuda:0")
    back = api.cq_background(0.1, -0.2, omega_m=0.3)
    prm = api.cq_model_params(box, a, 0.1, -0.2, omega_m=0.3, background=back)
    row = bg.interp(back[1], a)
    assert abs(prm.cq_phibar / row[3] - 1.0) < 1e-13 and prm.cq_lambda == back[0].lam
    P = oracle.params(oracle.CQ, n, box, a=a, omega_m=0.3, alpha=0.1, beta=-0.2,
                      phibar=row[3], lam=back[0].lam)
    d = synthetic.lognormal_delta(n, 77, sigma_delta=1.5).astype(np.float32)
    ref, _, rel, _ = oracle.solve(P, d.astype(np.float64), tol=1e-12)
    mg = api.Context(n, device=dev)
    field, st = mg.solve("cq", prm, torch.from_numpy(d).to(dev), tol=1e-9,
                         opts=api.solver_opts(precision="fp32"))
    err = np.linalg.norm(field.cpu().numpy() - ref) / np.linalg.norm(ref)
    print(f"a={a} phibar={row[3]:.4f} lambda={back[0].lam:.6f} cycles={st.cycles} err={err:.1e}",
          flush=True)
    assert err < 1e-5
    mg.close()
