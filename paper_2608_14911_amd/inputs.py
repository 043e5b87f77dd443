"""Seeded synthetic inputs for the short-range MD step.

This module holds no arithmetic of the method (no forces, no neighbour
search, no integration): it only draws starting states from seeds, so that the
FP64 oracle and the HIP library can be fed identical inputs.  All draws come
from numpy's Philox4x64-10 bit generator keyed by (seed, stream):

    stream 1: initial velocities      stream 2: positions / jitter
    stream 3: batch sampling          stream 4: network initialisation
    stream 5: minibatch order

The workloads mirror the paper's only concrete run (section "Example usage":
random positions in a periodic box, zero velocities, WCA with a capping
radius for push-off) and the standard LJ-fluid and Kremer-Grest-melt
benchmarks built on the same interactions.
"""
import math

import numpy as np

WCA_RC = 2.0 ** (1.0 / 6.0)

STREAM_VEL = 1
STREAM_POS = 2
STREAM_BATCH = 3
STREAM_MLP = 4
STREAM_MINIBATCH = 5


def rng(seed, stream):
    """numpy Generator on Philox4x64-10 with key (seed, stream)."""
    return np.random.Generator(np.random.Philox(key=np.array([seed, stream], dtype=np.uint64)))


def wrap_into_box(x, box):
    """Fold coordinates into [0, L) per dimension (input preparation)."""
    box = np.asarray(box, dtype=np.float64)
    y = np.mod(x, box)
    y = np.where(y >= box, 0.0, y)
    return np.ascontiguousarray(y, dtype=np.float64)


def fcc_lattice(ncell, density, jitter=0.0, seed=0):
    """FCC lattice of ncell^3 cubic cells (4 sites each) at number density
    ``density``; each coordinate jittered uniformly in [-jitter, jitter].
    Returns (pos [N,3] in [0,L), box [3])."""
    a = (4.0 / density) ** (1.0 / 3.0)
    L = ncell * a
    basis = np.array([[0.0, 0.0, 0.0], [0.5, 0.5, 0.0], [0.5, 0.0, 0.5], [0.0, 0.5, 0.5]])
    g = np.arange(ncell, dtype=np.float64)
    cz, cy, cx = np.meshgrid(g, g, g, indexing="ij")
    cells = np.stack([cx.ravel(), cy.ravel(), cz.ravel()], axis=1)
    pos = (cells[:, None, :] + basis[None, :, :]).reshape(-1, 3) * a
    if jitter > 0.0:
        pos = pos + rng(seed, STREAM_POS).uniform(-jitter, jitter, size=pos.shape)
    box = np.array([L, L, L])
    return wrap_into_box(pos, box), box


def maxwell_boltzmann(n, temperature, mass=1.0, seed=0, zero_momentum=True, exact=True, ndof=None):
    """Gaussian velocities N(0, kT/m); optionally remove the centre-of-mass
    velocity and rescale so that 2K/ndof equals ``temperature`` exactly
    (ndof defaults to 3N-3 when the momentum is removed, else 3N)."""
    m = np.broadcast_to(np.asarray(mass, dtype=np.float64), (n,))
    v = rng(seed, STREAM_VEL).standard_normal((n, 3)) * np.sqrt(temperature / m)[:, None]
    if zero_momentum:
        p = (m[:, None] * v).sum(axis=0) / m.sum()
        v = v - p[None, :]
    if exact and n > 1:
        if ndof is None:
            ndof = 3 * n - 3 if zero_momentum else 3 * n
        k2 = (m[:, None] * v * v).sum()
        v = v * math.sqrt(temperature * ndof / k2)
    return np.ascontiguousarray(v, dtype=np.float64)


def random_positions(n, box, seed=0):
    """Uniform random positions in the box (the paper's getRandomPos())."""
    box = np.asarray(box, dtype=np.float64)
    return wrap_into_box(rng(seed, STREAM_POS).uniform(0.0, 1.0, size=(n, 3)) * box, box)


def random_walk_chains(n_chains, chain_len, density, bond=0.97, seed=0):
    """Freely jointed chains: first bead uniform in the box, each next bead at
    distance ``bond`` in a uniformly random direction; no overlap rejection.
    Returns dict(pos, box, bonds [nb,2], angles [na,3], chain_len, n_chains)."""
    n = n_chains * chain_len
    L = (n / density) ** (1.0 / 3.0)
    box = np.array([L, L, L])
    g = rng(seed, STREAM_POS)
    first = g.uniform(0.0, L, size=(n_chains, 3))
    steps = g.standard_normal((n_chains, max(chain_len - 1, 0), 3))
    steps /= np.linalg.norm(steps, axis=2, keepdims=True)
    steps *= bond
    walk = np.concatenate([first[:, None, :], first[:, None, :] + np.cumsum(steps, axis=1)], axis=1)
    pos = wrap_into_box(walk.reshape(-1, 3), box)
    base = (np.arange(n_chains) * chain_len)[:, None]
    if chain_len >= 2:
        k = np.arange(chain_len - 1)[None, :]
        bonds = np.stack([(base + k).ravel(), (base + k + 1).ravel()], axis=1).astype(np.int32)
    else:
        bonds = np.zeros((0, 2), dtype=np.int32)
    if chain_len >= 3:
        k = np.arange(chain_len - 2)[None, :]
        angles = np.stack([(base + k).ravel(), (base + k + 1).ravel(), (base + k + 2).ravel()],
                          axis=1).astype(np.int32)
    else:
        angles = np.zeros((0, 3), dtype=np.int32)
    return {"pos": pos, "box": box, "bonds": bonds, "angles": angles,
            "chain_len": chain_len, "n_chains": n_chains}


def lattice_melt(n_chains, chain_len, density, jitter=0.05, seed=0):
    """Chains laid along a boustrophedon path through a simple cubic lattice
    (m^3 >= n sites, spacing a = (n / density)^(1/3) / m), cut into
    ``n_chains`` consecutive pieces of ``chain_len`` beads, with uniform
    jitter +-``jitter``*a per component (stream 2).  Bonds join lattice
    neighbours (length a), so no bead overlaps and no push-off is needed.
    Returns dict(pos, box, bonds, angles, chain_len, n_chains)."""
    n = n_chains * chain_len
    m = int(np.ceil(n ** (1.0 / 3.0) - 1e-9))
    L = (n / density) ** (1.0 / 3.0)
    a = L / m
    # boustrophedon order: x reverses on odd rows, y on odd planes, so that
    # consecutive sites are lattice neighbours
    iz, j, i = np.meshgrid(np.arange(m), np.arange(m), np.arange(m), indexing="ij")
    iy = np.where(iz % 2 == 1, m - 1 - j, j)          # j-th row visited in plane iz
    ix = np.where((iz * m + j) % 2 == 1, m - 1 - i, i)  # direction alternates with every row
    sites = np.stack([ix.ravel(), iy.ravel(), iz.ravel()], axis=1)[:n].astype(np.float64)
    g = rng(seed, STREAM_POS)
    pos = (sites + 0.5 + g.uniform(-jitter, jitter, size=(n, 3))) * a
    box = np.array([L, L, L])
    pos = wrap_into_box(pos, box)
    base = (np.arange(n_chains) * chain_len)[:, None]
    k = np.arange(chain_len - 1)[None, :]
    bonds = np.stack([(base + k).ravel(), (base + k + 1).ravel()], axis=1).astype(np.int32)
    k = np.arange(chain_len - 2)[None, :]
    angles = np.stack([(base + k).ravel(), (base + k + 1).ravel(), (base + k + 2).ravel()], axis=1).astype(np.int32)
    return {"pos": pos, "box": box, "bonds": bonds, "angles": angles,
            "chain_len": chain_len, "n_chains": n_chains}


# ------------------------------------------------------------------ workloads
def kg_params(rc=WCA_RC, fene_K=30.0, fene_R0=1.5, k_bend=0.0):
    return {"eps": 1.0, "sigma": 1.0, "rc": rc, "shift": float("nan"), "caprad": 0.0,
            "fene_K": fene_K, "fene_R0": fene_R0, "k_bend": k_bend}


def workload_kg1k(seed=1000):
    """20 chains x 50 beads at density 0.85, WCA + FENE (K=30, R0=1.5),
    Langevin T=1, gamma=1, dt=0.01, skin 0.3; MB velocities at T=1."""
    w = random_walk_chains(20, 50, 0.85, bond=0.97, seed=seed)
    w["vel"] = maxwell_boltzmann(w["pos"].shape[0], 1.0, seed=seed, zero_momentum=False, exact=False)
    w.update(kg_params(k_bend=0.0))
    w.update({"dt": 0.01, "skin": 0.3, "temperature": 1.0, "gamma": 1.0, "integrator": "langevin",
              "seed": seed, "name": "KG melt 20x50 (1,000 beads), WCA+FENE, Langevin"})
    return w


def workload_lj(ncell=64, seed=1001, jitter=0.05):
    """LJ fluid: FCC start (4*ncell^3 sites) at density 0.8442 with uniform
    jitter, T=0.72, rc=2.5 shifted, skin 0.3, NVE dt=0.005."""
    pos, box = fcc_lattice(ncell, 0.8442, jitter=jitter, seed=seed)
    n = pos.shape[0]
    vel = maxwell_boltzmann(n, 0.72, seed=seed, zero_momentum=True, exact=True)
    return {"pos": pos, "box": box, "vel": vel, "bonds": None, "angles": None,
            "eps": 1.0, "sigma": 1.0, "rc": 2.5, "shift": float("nan"), "caprad": 0.0,
            "dt": 0.005, "skin": 0.3, "temperature": 0.72, "gamma": 0.0, "integrator": "nve",
            "seed": seed, "name": "LJ fluid %d particles (FCC %d^3), rho 0.8442" % (n, ncell)}


def workload_kg(n_chains=2000, chain_len=1000, seed=1002):
    """Kremer-Grest melt: n_chains x chain_len random walks at density 0.85,
    WCA + FENE (K=30, R0=1.5) + cosine bending k=1.5, Langevin T=1,
    gamma=0.5, dt=0.01, skin 0.4."""
    w = random_walk_chains(n_chains, chain_len, 0.85, bond=0.97, seed=seed)
    w["vel"] = maxwell_boltzmann(w["pos"].shape[0], 1.0, seed=seed, zero_momentum=False, exact=False)
    w.update(kg_params(k_bend=1.5))
    w.update({"dt": 0.01, "skin": 0.4, "temperature": 1.0, "gamma": 0.5, "integrator": "langevin",
              "seed": seed, "name": "KG melt %dx%d, WCA+FENE+bending, Langevin" % (n_chains, chain_len)})
    return w


def workload_paper_example(n=10000, seed=1005):
    """The paper's example script: N=10,000 random positions in a 20^3 box,
    zero velocities, WCA (rc 1.12246) capped at 0.8, skin 0.3, Langevin
    gamma=1, T=1, warm-up dt 1e-4 then dt 0.005."""
    box = np.array([20.0, 20.0, 20.0])
    pos = random_positions(n, box, seed=seed)
    return {"pos": pos, "box": box, "vel": np.zeros((n, 3)), "bonds": None, "angles": None,
            "eps": 1.0, "sigma": 1.0, "rc": 1.12246, "shift": float("nan"), "caprad": 0.8,
            "dt": 0.0001, "skin": 0.3, "temperature": 1.0, "gamma": 1.0, "integrator": "langevin",
            "seed": seed, "name": "paper example, 10,000 particles, box 20^3"}


def mlp_init(seed=1004, n_in=32, hidden=64):
    """He-uniform initial weights of the 32 -> 64 -> 64 -> 1 network, biases
    zero, drawn from stream 4; FP64 vector in the layout W1 (hidden x n_in,
    row-major), b1, W2 (hidden x hidden), b2, w3 (hidden), b3."""
    g = rng(seed, 4)
    W1 = g.uniform(-1.0, 1.0, size=(hidden, n_in)) * np.sqrt(6.0 / n_in)
    W2 = g.uniform(-1.0, 1.0, size=(hidden, hidden)) * np.sqrt(6.0 / hidden)
    w3 = g.uniform(-1.0, 1.0, size=hidden) * np.sqrt(6.0 / hidden)
    return np.concatenate([W1.ravel(), np.zeros(hidden), W2.ravel(), np.zeros(hidden), w3, np.zeros(1)])


def batch_replicas(nsys=256, seed=1003, n_min=2048, n_max=65536):
    """Replicas of uneven size for a batch.  From stream 3 of ``seed``, per
    replica r: N = round(exp(U[ln n_min, ln n_max])), density U[0.70, 0.90],
    temperature U[0.7, 1.2], and for the melts a chain length U{10..200}.
    Even r: LJ fluid (rc 2.5 shifted, NVE, dt 0.005, skin 0.3) started from a
    random subset of ceil((N/4)^(1/3))^3 * 4 FCC sites rescaled to the
    density, jitter 0.05.  Odd r: Kremer-Grest melt (WCA + FENE + bending
    1.5, Langevin gamma 0.5, dt 0.01, skin 0.4) of round(N / L_c) random
    walks (raw: a push-off is needed).  Each replica's own positions and
    velocities come from seed 100000 * seed + r (streams 1 and 2)."""
    g = rng(seed, STREAM_BATCH)
    out = []
    for r in range(nsys):
        n = int(round(math.exp(g.uniform(math.log(n_min), math.log(n_max)))))
        rho = float(g.uniform(0.70, 0.90))
        temp = float(g.uniform(0.7, 1.2))
        lc = int(g.integers(10, 201))
        sub = 100000 * seed + r
        if r % 2 == 0:
            nc = int(math.ceil((n / 4.0) ** (1.0 / 3.0)))
            L = (n / rho) ** (1.0 / 3.0)
            sites, _ = fcc_lattice(nc, 4.0 * nc ** 3 / L ** 3)
            gp = rng(sub, STREAM_POS)
            pick = gp.choice(sites.shape[0], size=n, replace=False)
            pos = sites[np.sort(pick)] + gp.uniform(-0.05, 0.05, size=(n, 3))
            box = np.array([L, L, L])
            out.append({"kind": "lj", "pos": wrap_into_box(pos, box), "box": box,
                        "vel": maxwell_boltzmann(n, temp, seed=sub), "bonds": None, "angles": None,
                        "pair": {(0, 0): (1.0, 1.0, 2.5, float("nan"), 0.0)}, "dt": 0.005, "skin": 0.3,
                        "integrator": "nve", "temperature": temp, "gamma": 0.0, "seed": sub, "k_bend": 0.0,
                        "density": rho})
        else:
            nch = max(1, int(round(n / lc)))
            w = random_walk_chains(nch, lc, rho, bond=0.97, seed=sub)
            n = nch * lc
            out.append({"kind": "kg", "pos": w["pos"], "box": w["box"],
                        "vel": maxwell_boltzmann(n, temp, seed=sub, zero_momentum=False, exact=False),
                        "bonds": w["bonds"], "angles": w["angles"],
                        "pair": {(0, 0): (1.0, 1.0, WCA_RC, float("nan"), 0.0)}, "dt": 0.01, "skin": 0.4,
                        "integrator": "langevin", "temperature": temp, "gamma": 0.5, "seed": sub, "k_bend": 1.5,
                        "density": rho, "chain_len": lc})
    return out
