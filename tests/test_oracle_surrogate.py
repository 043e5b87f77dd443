"""Pins of the FP64 surrogate oracle against mathematics: closed forms of the
basis, finite differences of the energy (forces) and of the loss (parameter
gradient), Newton's third law, translation invariance, the reduction of a
constant input gradient to a pair potential, and Adam's first step."""
import numpy as np
import pytest

from oracle import surrogate as S
from paper_2608_14911_amd import inputs


def rand_theta(seed, scale=1.0, bias=0.3):
    th = inputs.mlp_init(seed) * scale
    g = np.random.default_rng(seed)
    for lo, hi in ((S.O_B1, S.O_W2), (S.O_B2, S.O_W3), (S.O_B3, S.NPARAM)):
        th[lo:hi] = g.uniform(-bias, bias, size=hi - lo)
    return th


def small_system(seed, n=40, L=6.0, dmin=0.8):
    g = np.random.default_rng(seed)
    pts = []
    while len(pts) < n:
        p = g.uniform(0, L, size=3)
        ok = True
        for q in pts:
            d = p - q
            d -= L * np.round(d / L)
            if d @ d < dmin * dmin:
                ok = False
                break
        if ok:
            pts.append(p)
    return np.array(pts), np.array([L, L, L])


def norm_consts(pos, box):
    G = S.descriptors(pos, box)
    return G.mean(0), 1.0 / (G.std(0) + 1e-3)


def test_layout_and_centres():
    assert S.NPARAM == 6337
    mu = S.centres()
    assert mu[0] == 0.8 and abs(mu[-1] - 2.5) < 1e-15
    assert np.allclose(np.diff(mu), 1.7 / 31)


def test_basis_closed_forms_and_derivative():
    mu = S.centres()
    rd = S.RD
    g, dg = S.basis(mu)
    fc = 0.5 * (np.cos(np.pi * mu / rd) + 1.0)
    assert np.allclose(np.diag(g), fc, rtol=0, atol=1e-15)      # phi_k(mu_k) = 1
    # value and slope vanish at the cutoff
    g, dg = S.basis(np.array([rd]))
    assert np.abs(g).max() < 1e-30 and np.abs(dg).max() < 1e-12
    # one basis function in closed form at an arbitrary r
    r = 1.234
    phi3 = np.exp(-(r - mu[3]) ** 2 / 0.02)
    assert abs(S.basis(r)[0][3] - phi3 * 0.5 * (np.cos(np.pi * r / rd) + 1)) < 1e-16
    rs = np.linspace(0.7, 2.49, 41)
    h = 1e-6
    fd = (S.basis(rs + h)[0] - S.basis(rs - h)[0]) / (2 * h)
    assert np.abs(fd - S.basis(rs)[1]).max() < 1e-6


def test_silu_derivatives():
    z = np.linspace(-6, 6, 61)
    h = 1e-5
    assert np.abs((S.silu(z + h) - S.silu(z - h)) / (2 * h) - S.dsilu(z)).max() < 1e-9
    assert np.abs((S.dsilu(z + h) - S.dsilu(z - h)) / (2 * h) - S.d2silu(z)).max() < 1e-9


def test_descriptor_two_and_three_particles():
    box = np.array([8.0, 8.0, 8.0])
    pos = np.array([[1.0, 1.0, 1.0], [2.3, 1.0, 1.0], [1.0, 1.0, 3.6]])   # third at 2.6 > r_d from the first
    G = S.descriptors(pos, box)
    g01 = S.basis(1.3)[0]
    r12 = np.hypot(1.3, 2.6)
    assert r12 > S.RD
    assert np.allclose(G[0], g01, atol=1e-16) and np.allclose(G[1], g01, atol=1e-16)
    assert np.abs(G[2]).max() == 0.0
    # periodic image across the boundary counts the same
    pos2 = np.array([[0.2, 4.0, 4.0], [7.7, 4.0, 4.0]])
    G2 = S.descriptors(pos2, box)
    assert np.allclose(G2[0], S.basis(0.5)[0], atol=1e-15)


def test_standardisation_fcc_and_two_point():
    # a perfect FCC crystal: every particle sees the same shells (12 at the
    # nearest-neighbour distance d, then 6 at d sqrt 2, 24 at d sqrt 3 and 12
    # at 2d; the next shell, d sqrt 5, lies beyond r_d at density 0.85), so
    # every row equals the shell sum and the variance vanishes
    nc, rho = 4, 0.85
    a = (4.0 / rho) ** (1.0 / 3.0)
    base = np.array([[0, 0, 0], [0.5, 0.5, 0], [0.5, 0, 0.5], [0, 0.5, 0.5]])
    cells = np.array([[i, j, k] for i in range(nc) for j in range(nc) for k in range(nc)], dtype=float)
    pos = ((cells[:, None, :] + base[None]) * a).reshape(-1, 3)
    box = np.full(3, nc * a)
    d = a / np.sqrt(2.0)
    assert d * np.sqrt(5.0) > S.RD > 2.0 * d
    shells = 12 * S.basis(d)[0] + 6 * S.basis(d * np.sqrt(2))[0] + 24 * S.basis(d * np.sqrt(3))[0] \
        + 12 * S.basis(2 * d)[0]
    m, istd = S.standardisation([pos, pos + 0.37], box)
    assert np.allclose(m, shells, rtol=1e-13, atol=1e-15)
    assert np.allclose(istd, 1.0 / np.sqrt(1e-6), rtol=1e-6)
    # two frames of one isolated pair at r0 and r1: the rows take two values
    # with equal weight, so the mean is their midpoint and the variance the
    # square of half their difference
    box = np.full(3, 20.0)
    r0, r1 = 1.05, 1.6
    f0 = np.array([[5.0, 5.0, 5.0], [5.0 + r0, 5.0, 5.0]])
    f1 = np.array([[5.0, 5.0, 5.0], [5.0, 5.0 + r1, 5.0]])
    m, istd = S.standardisation([f0, f1], box)
    b0, b1 = S.basis(r0)[0], S.basis(r1)[0]
    assert np.allclose(m, 0.5 * (b0 + b1), rtol=0, atol=1e-15)
    assert np.allclose(istd, 1.0 / np.sqrt((0.5 * (b0 - b1)) ** 2 + 1e-6), rtol=1e-12)


@pytest.mark.parametrize("seed", [0, 1])
def test_forces_are_minus_energy_gradient(seed):
    pos, box = small_system(seed)
    m, istd = norm_consts(pos, box)
    th = rand_theta(seed)
    E, Ei, F, a, W = S.energy_forces(th, m, istd, pos, box)
    h = 1e-6
    fd = np.zeros_like(F)
    for i in range(pos.shape[0]):
        for d in range(3):
            p = pos.copy(); p[i, d] += h
            ep = S.energy_forces(th, m, istd, p, box)[0]
            p[i, d] -= 2 * h
            em = S.energy_forces(th, m, istd, p, box)[0]
            fd[i, d] = -(ep - em) / (2 * h)
    assert np.linalg.norm(fd - F) / np.linalg.norm(F) < 1e-7
    # Newton's third law and translation invariance
    assert np.abs(F.sum(0)).max() < 1e-12 * np.abs(F).sum()
    shift = np.array([0.37, -1.1, 2.9])
    E2, _, F2, _, W2 = S.energy_forces(th, m, istd, (pos + shift) % box, box)
    assert abs(E2 - E) < 1e-12 * abs(E) and np.abs(F2 - F).max() < 1e-10 * np.abs(F).max()
    # virial from the pair decomposition equals -sum x.F for a box-free
    # cluster (the same particles placed far from every periodic image)
    big = np.array([40.0, 40.0, 40.0])
    cl = pos.copy()
    cl -= cl.mean(0)
    E3, _, F3, _, W3 = S.energy_forces(th, m, istd, cl + 20.0, big)
    assert abs(W3 - float((cl * F3).sum())) < 1e-9 * np.abs(cl * F3).sum()


def test_constant_input_gradient_is_a_pair_potential():
    """a_i = c for every particle makes E a pair potential
    u(r) = 2 c . g(r) per unordered pair (each pair enters G(i) and G(j));
    its forces are -u'(r) along the pair, written here with u' by central
    differences of the closed-form basis."""
    pos, box = small_system(3, n=30)
    c = np.random.default_rng(3).normal(size=32)
    a = np.tile(c, (pos.shape[0], 1))
    F, W = S.pair_forces(a, pos, box)
    mu = S.centres()

    def u(r):
        phi = np.exp(-(r - mu) ** 2 / (2 * 0.1 ** 2))
        return 2.0 * float(c @ (phi * 0.5 * (np.cos(np.pi * r / 2.5) + 1.0)))

    n = pos.shape[0]
    Fr = np.zeros_like(F)
    Wr = 0.0
    h = 1e-6
    for i in range(n):
        for j in range(i + 1, n):
            d = pos[j] - pos[i]
            d -= box * np.round(d / box)
            r = np.sqrt(d @ d)
            if r >= 2.5:
                continue
            du = (u(r + h) - u(r - h)) / (2 * h)
            Fr[i] += du * d / r        # -u'(r) * (x_i - x_j)/r
            Fr[j] -= du * d / r
            Wr += -du * r
    assert np.abs(F - Fr).max() < 1e-7 * np.abs(Fr).max()
    assert abs(W - Wr) < 1e-7 * abs(Wr)


@pytest.mark.parametrize("seed", [0, 5])
def test_loss_gradient_matches_finite_differences(seed):
    pos0, box = small_system(seed, n=24)
    g = np.random.default_rng(seed + 100)
    frames = [pos0, (pos0 + g.normal(scale=0.05, size=pos0.shape)) % box]
    f_ref = [g.normal(size=pos0.shape) * 3.0 for _ in frames]
    m, istd = norm_consts(pos0, box)
    th = rand_theta(seed)
    loss, grad = S.loss_grad(th, m, istd, frames, f_ref, box)
    assert grad[S.O_B3] == 0.0
    idx = np.concatenate([g.choice(S.NPARAM - 1, size=60, replace=False),
                          [S.O_W3, S.O_W3 + 7, S.O_B2 + 3, S.O_B1 + 11, S.O_B3]])
    fd = np.zeros(len(idx))
    for q, k in enumerate(idx):
        h = 1e-5 * max(1.0, abs(th[k]))
        tp = th.copy(); tp[k] += h
        tm = th.copy(); tm[k] -= h
        fd[q] = (S.loss_grad(tp, m, istd, frames, f_ref, box, with_grad=False)[0] -
                 S.loss_grad(tm, m, istd, frames, f_ref, box, with_grad=False)[0]) / (2 * h)
    assert np.linalg.norm(fd - grad[idx]) / np.linalg.norm(fd) < 1e-6
    # loss definition: mean of squared force residuals
    F0 = S.energy_forces(th, m, istd, frames[0], box)[2]
    F1 = S.energy_forces(th, m, istd, frames[1], box)[2]
    ref = (((F0 - f_ref[0]) ** 2).sum() + ((F1 - f_ref[1]) ** 2).sum()) / (2 * 3 * 24)
    assert abs(loss - ref) < 1e-12 * ref


def test_adam_first_step_and_schedule():
    g = np.array([0.5, -2.0, 1e-3, 0.0])
    th = np.array([1.0, 1.0, 1.0, 1.0])
    z = np.zeros(4)
    t1, m1, m2 = S.adam_step(th, z, z, g, 1, 1e-3)
    assert np.allclose(t1, th - 1e-3 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    assert np.allclose(m1, 0.1 * g) and np.allclose(m2, 0.001 * g * g)
    assert S.cosine_lr(0, 100, 1e-3) == 1e-3
    assert abs(S.cosine_lr(50, 100, 1e-3) - 5e-4) < 1e-18
