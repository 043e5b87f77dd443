"""FP64 oracle of the learned non-bonded surrogate (plain numpy).

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle/``: only ``tests/``,
``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may
import it.  It shares no code with the HIP library.

The paper names the model only in outline (a per-particle descriptor of 32
Gaussian radial basis functions of width 0.1 with centres from 0.8 to 2.5,
an MLP 32 -> 64 -> 64 -> 1 with SiLU giving a per-particle energy, forces from
its gradient, force-matching training).  The readings taken here:

* basis  phi_k(r) = exp(-(r - mu_k)^2 / (2 w^2)), w = 0.1, mu_k = 0.8 + k 1.7/31
  (k = 0..31, both ends included), times the cosine cutoff
  f_c(r) = (cos(pi r / r_d) + 1) / 2 with r_d = 2.5, so that the forces are
  continuous at r_d;  g_k(r) = phi_k(r) f_c(r);
* descriptor  G_k(i) = sum over j != i with r_ij < r_d of g_k(r_ij);
* standardisation  x_i = (G(i) - m) * istd with fixed training-set
  constants, not trained: m and istd = 1 / sqrt(var + 1e-6) per basis
  function over all descriptor rows of the training frames (population
  variance; the floor keeps functions with almost no signal finite);
* E_i = w3 . silu(W2 silu(W1 x_i + b1) + b2) + b3,  E = sum_i E_i,
  F_i = -dE/dr_i;
* parameter vector theta (6,337 values) = W1 (64x32 row-major), b1 (64),
  W2 (64x64), b2 (64), w3 (64), b3 (1);
* loss  L = mean over frames, particles and components of (F - F_ref)^2;
* Adam (Kingma and Ba 2015) with bias correction, and a cosine learning-rate
  decay lr_t = lr0 (1 + cos(pi t / T)) / 2.

Every function below is the plain definition written out; the gradient of
the loss is the analytic double backward derived from these definitions.
"""
import math

import numpy as np

NB = 32
H = 64
WIDTH = 0.1
MU0, MU1 = 0.8, 2.5
RD = 2.5

# parameter layout
O_W1 = 0
O_B1 = O_W1 + H * NB
O_W2 = O_B1 + H
O_B2 = O_W2 + H * H
O_W3 = O_B2 + H
O_B3 = O_W3 + H
NPARAM = O_B3 + 1


def centres():
    return np.array([MU0 + k * (MU1 - MU0) / (NB - 1) for k in range(NB)])


def unpack(theta):
    t = np.asarray(theta, dtype=np.float64)
    assert t.shape == (NPARAM,)
    return (t[O_W1:O_B1].reshape(H, NB), t[O_B1:O_W2], t[O_W2:O_B2].reshape(H, H), t[O_B2:O_W3],
            t[O_W3:O_B3], t[O_B3])


def pack(W1, b1, W2, b2, w3, b3):
    return np.concatenate([np.ravel(W1), b1, np.ravel(W2), b2, w3, np.atleast_1d(b3)]).astype(np.float64)


def basis(r, rd=RD):
    """g_k(r) and dg_k/dr for r < rd (shape [..., 32])."""
    r = np.asarray(r, dtype=np.float64)[..., None]
    mu = centres()
    phi = np.exp(-(r - mu) ** 2 / (2.0 * WIDTH * WIDTH))
    dphi = -(r - mu) / (WIDTH * WIDTH) * phi
    fc = 0.5 * (np.cos(np.pi * r / rd) + 1.0)
    dfc = -0.5 * np.pi / rd * np.sin(np.pi * r / rd)
    return phi * fc, dphi * fc + phi * dfc


def pairs(pos, box, rd=RD):
    """Ordered pairs (i, j), j != i, r_ij < rd: arrays I, J, D = x_j - x_i
    (minimum image, compare-based) and r = |D|.  Brute force over all pairs
    in row blocks; the box must be at least 2 rd per side."""
    pos = np.asarray(pos, dtype=np.float64)
    L = np.asarray(box, dtype=np.float64)
    assert np.all(L >= 2.0 * rd)
    n = pos.shape[0]
    Is, Js, Ds = [], [], []
    blk = max(1, 2_000_000 // max(n, 1))
    for a in range(0, n, blk):
        b = min(n, a + blk)
        d = pos[None, :, :] - pos[a:b, None, :]
        d = np.where(d > 0.5 * L, d - L, d)
        d = np.where(d < -0.5 * L, d + L, d)
        r2 = (d * d).sum(-1)
        ii, jj = np.nonzero(r2 < rd * rd)
        keep = (ii + a) != jj
        ii, jj = ii[keep], jj[keep]
        Is.append(ii + a)
        Js.append(jj)
        Ds.append(d[ii, jj])
    I = np.concatenate(Is)
    J = np.concatenate(Js)
    D = np.concatenate(Ds) if Ds else np.zeros((0, 3))
    return I, J, D, np.sqrt((D * D).sum(-1))


def descriptors(pos, box, rd=RD, pr=None):
    I, J, D, r = pr if pr is not None else pairs(pos, box, rd)
    g, _ = basis(r, rd)
    G = np.zeros((np.asarray(pos).shape[0], NB))
    np.add.at(G, I, g)
    return G


def standardisation(frames, box, rd=RD, floor=1e-6):
    """The fixed standardisation constants (m, istd) of the network input:
    mean and 1/sqrt(var + floor) of each descriptor component over every
    particle of every frame."""
    G = np.concatenate([descriptors(f, box, rd) for f in frames])
    m = G.mean(0)
    var = ((G - m) ** 2).mean(0)
    return m, 1.0 / np.sqrt(var + floor)


def silu(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return z * s


def dsilu(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def d2silu(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 - s) * (2.0 + z * (1.0 - 2.0 * s))


def mlp(theta, x):
    """Per-particle energies E [P] and input gradients dE/dx [P, 32]."""
    W1, b1, W2, b2, w3, b3 = unpack(theta)
    z1 = x @ W1.T + b1
    h1 = silu(z1)
    z2 = h1 @ W2.T + b2
    h2 = silu(z2)
    E = h2 @ w3 + b3
    gz2 = w3 * dsilu(z2)
    gz1 = (gz2 @ W2) * dsilu(z1)
    return E, gz1 @ W1


def energy_forces(theta, m, istd, pos, box, rd=RD, want_fscale=False):
    """Surrogate energy E = sum_i E_i, per-particle E_i, forces F = -dE/dr,
    the per-particle input gradients a_i = dE_i/dG(i), and the virial
    W = sum over unordered pairs of r_ij . f_ij (the model is radial, so the
    force splits into central pair terms).  With want_fscale, also
    sum_j |f_ij| per particle (the scale of the cancellation in F_i)."""
    pr = pairs(pos, box, rd)
    G = descriptors(pos, box, rd, pr)
    x = (G - m) * istd
    Ei, gx = mlp(theta, x)
    a = gx * istd
    out = pair_forces(a, pos, box, rd, pr, want_fscale)
    return (float(Ei.sum()), Ei) + (out[0], a) + out[1:]


def pair_forces(a, pos, box, rd=RD, pr=None, want_fscale=False):
    """Forces of E = sum_i E_i(G(i)) given a_i = dE_i/dG(i):
    F_i = sum_j c_ij (x_j - x_i) / r_ij with c_ij = (a_i + a_j) . g'(r_ij),
    and the virial W = -1/2 sum over ordered pairs of c_ij r_ij."""
    I, J, D, r = pr if pr is not None else pairs(pos, box, rd)
    _, dg = basis(r, rd)
    c = ((a[I] + a[J]) * dg).sum(-1)
    n = np.asarray(pos).shape[0]
    F = np.zeros((n, 3))
    np.add.at(F, I, (c / r)[:, None] * D)
    W = 0.5 * float((-c * r).sum())
    if not want_fscale:
        return F, W
    fs = np.zeros(n)
    np.add.at(fs, I, np.abs(c))
    return F, W, fs


def loss_grad(theta, m, istd, frames, f_ref, box, rd=RD, with_grad=True):
    """Force-matching loss over frames and its analytic gradient.

    With delta_i = dL/dF_i = 2 (F_i - F_ref,i) / M and D_ij = x_j - x_i,
        dL/dtheta = sum_p u_p . da_p/dtheta,
        u_p = sum_j ((delta_p - delta_j) . D_pj / r_pj) g'(r_pj),
    and u_p . a_p = v_p . dE_p/dx_p with v_p = u_p * istd.  The derivative of
    s_p = v_p . dE_p/dx_p with v_p held fixed is the double backward: a
    forward tangent t1 = W1 v, t2 = W2 (silu'(z1) t1), then
        ds/dw3 = silu'(z2) t2,            ds/db3 = 0,
        r2 = w3 silu''(z2) t2,            gz2 = w3 silu'(z2),
        ds/dW2 = r2 h1^T + gz2 (silu'(z1) t1)^T,   ds/db2 = r2,
        gh1 = W2^T gz2,
        r1 = (W2^T r2) silu'(z1) + gh1 t1 silu''(z1),   gz1 = gh1 silu'(z1),
        ds/dW1 = r1 x^T + gz1 v^T,        ds/db1 = r1.
    """
    W1, b1, W2, b2, w3, b3 = unpack(theta)
    nf = len(frames)
    n = np.asarray(frames[0]).shape[0]
    M = 3.0 * n * nf
    loss = 0.0
    grad = np.zeros(NPARAM)
    for f in range(nf):
        pos = np.asarray(frames[f], dtype=np.float64)
        pr = pairs(pos, box, rd)
        I, J, D, r = pr
        G = descriptors(pos, box, rd, pr)
        x = (G - m) * istd
        z1 = x @ W1.T + b1
        h1 = silu(z1)
        z2 = h1 @ W2.T + b2
        gz2 = w3 * dsilu(z2)
        gh1 = gz2 @ W2
        gz1 = gh1 * dsilu(z1)
        a = (gz1 @ W1) * istd
        _, dg = basis(r, rd)
        c = ((a[I] + a[J]) * dg).sum(-1)
        F = np.zeros((n, 3))
        np.add.at(F, I, (c / r)[:, None] * D)
        res = F - np.asarray(f_ref[f], dtype=np.float64)
        loss += float((res * res).sum()) / M
        if not with_grad:
            continue
        delta = 2.0 * res / M
        proj = ((delta[I] - delta[J]) * D).sum(-1) / r
        u = np.zeros((n, NB))
        np.add.at(u, I, proj[:, None] * dg)
        v = u * istd
        t1 = v @ W1.T
        st1 = dsilu(z1) * t1
        t2 = st1 @ W2.T
        r2 = w3 * d2silu(z2) * t2
        r1 = (r2 @ W2) * dsilu(z1) + gh1 * t1 * d2silu(z1)
        g = unpack(grad)
        g[0][...] += r1.T @ x + gz1.T @ v
        g[1][...] += r1.sum(0)
        g[2][...] += r2.T @ h1 + gz2.T @ st1
        g[3][...] += r2.sum(0)
        g[4][...] += (dsilu(z2) * t2).sum(0)
    return loss, grad


def adam_step(theta, m1, m2, g, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update at step t >= 1 (bias-corrected); returns new arrays."""
    m1 = beta1 * m1 + (1.0 - beta1) * g
    m2 = beta2 * m2 + (1.0 - beta2) * g * g
    mh = m1 / (1.0 - beta1 ** t)
    vh = m2 / (1.0 - beta2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m1, m2


def cosine_lr(t, total, lr0):
    """Learning rate of update t (0-based) out of total."""
    return lr0 * 0.5 * (1.0 + math.cos(math.pi * t / total))
