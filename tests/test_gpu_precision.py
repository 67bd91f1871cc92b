"""Precision mode: an FP32 ground vector refined in FP64 (the caller's start
vector option of edx_lanczos_ground_state), against the FP64 oracle.

Bars: the refined E0 within 1e-10 relative of the oracle (the FP64 bar), in
fewer Lanczos steps than the FP64 solve from the random start vector; the
refined psi0's FP64 residual |H psi - E psi| below the FP32 one; G of the
refined vector (FP64 Krylov vectors) within 1e-8 max|G| of the exact Lehmann
sum.  A zero start vector is refused (EDX_E_INVALID); a start vector is
replayed exactly (psi0 bit for bit the same in two calls)."""
import numpy as np
import pytest

from oracle import fock, green, spectra
from paper_2105_06806_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def edx():
    import torch
    from paper_2105_06806_amd import edx as E
    assert torch.cuda.is_available()
    return E


def _resid(edx, S, psi, e):
    """|H psi - e psi| / |psi| with the FP64 product (psi cast to FP64)."""
    import torch
    x = psi.double()
    y = torch.empty_like(x)
    edx.hv(S, x, y)
    return float((y - e * x).norm() / x.norm())


def test_fp64_refinement_of_fp32_ground_vector(edx):
    import torch
    m, [sec] = inputs.workload("ns8")
    H = fock.explicit_hamiltonian(m, *sec)
    w, V = spectra.dense_lowest(H)
    S = edx.build_sector(m, *sec)
    e32, p32, r32, _ = edx.lanczos_ground_state(S, vtype="f32", niter=300, tol=1e-9, seed=3,
                                                allow=(edx.EDX_E_NOCONV,))
    e64, p64, r64, _ = edx.lanczos_ground_state(S, niter=300, tol=1e-14, rtol=1e-10, seed=3)
    start = p32.double().contiguous()
    ef, pf, rf, _ = edx.lanczos_ground_state(S, niter=300, tol=1e-14, rtol=1e-10, seed=3, start=start)
    assert abs(ef - w[0]) <= 1e-10 * abs(w[0])
    assert rf["iters"] < r64["iters"], (rf["iters"], r64["iters"])
    res32, resf = _resid(edx, S, p32, e32), _resid(edx, S, pf, ef)
    assert resf < res32 * 1e-2, (res32, resf)
    assert abs(abs(float(pf.cpu().numpy() @ V[:, 0])) - 1) < 1e-10
    beta, lm = 50.0, 128
    z = 1j * green.matsubara(beta, lm)
    G, _ = edx.green_cf(S, pf, ef, 0, 0, ngf=200, beta=beta, lmats=lm)
    Gl, _ = green.lehmann_exact(m, *sec, 0, 0, z)
    assert np.abs(G - Gl).max() <= 1e-8 * np.abs(Gl).max()


def test_start_vector_replay_and_refusal(edx):
    import torch
    m, [sec] = inputs.workload("ns8")
    S = edx.build_sector(m, *sec)
    gen = torch.Generator(device="cuda").manual_seed(4)
    start = torch.rand(S.dim, dtype=torch.float64, device="cuda", generator=gen) - 0.5
    a = edx.lanczos_ground_state(S, niter=200, tol=1e-13, seed=1, start=start)
    b = edx.lanczos_ground_state(S, niter=200, tol=1e-13, seed=99, start=start)   # seed unused
    assert a[0] == b[0] and bool(torch.equal(a[1], b[1]))
    with pytest.raises(edx.EdxError) as ei:
        edx.lanczos_ground_state(S, niter=50, start=torch.zeros_like(start))
    assert ei.value.status == edx.EDX_E_INVALID
    with pytest.raises(ValueError):
        edx.lanczos_ground_state(S, niter=50, start=start.float())
