"""Small seeded problems shared by the oracle pins and the GPU parity tests."""
import numpy as np

from oracle.layout import make_layout
from oracle.solver import Problem


def random_psfs(G_y, G_x, P, seed, positive=True):
    """Asymmetric random PSFs (non-negative, unit sum) so flips and
    transposes show up."""
    rng = np.random.default_rng(seed)
    h = rng.random((G_y, G_x, P, P)) ** 3
    if not positive:
        h = rng.standard_normal((G_y, G_x, P, P))
        return h
    return h / h.sum(axis=(2, 3), keepdims=True)


def tiny_problem(M=12, T=2, p=6, o=2, P=3, G=2, seed=0, model="interp", lam=1e-2,
                 reg="tv", reg_param=0.05, gamma=0.5, positivity=True, bc="neumann",
                 W_random=True, M_x=None, T_x=None, G_x=None, kind="pitch"):
    L = make_layout(M, T, p, o, P, G, model=model, M_x=M_x, T_x=T_x, G_x=G_x, kind=kind)
    rng = np.random.default_rng(seed + 100)
    psfs = random_psfs(L.ay.G, L.ax.G, P, seed)
    My, Mx = L.ay.M, L.ax.M
    y = rng.random((My, Mx)) + 0.1
    W = (0.5 + rng.random((My, Mx))) if W_random else np.ones((My, Mx))
    return Problem(L, psfs, y, W, lam=lam, reg=reg, reg_param=reg_param, gamma=gamma,
                   positivity=positivity, bc=bc)


def sharpening_network(kappa=0.5, theta=0.5):
    """out = x + kappa relu(Lap(x) - theta), Lap the 3 x 3 kernel 1 - (mean of
    the 8 neighbours): with kappa > 0 peaks are sharpened, with kappa < 0
    softened; smooth regions pass unchanged.  Every weight is exact in bf16."""
    P = [(np.zeros((32, 1, 3, 3)), np.zeros(32)), (np.zeros((32, 32, 3, 3)), np.zeros(32)),
         (np.zeros((32, 32, 3, 3)), np.zeros(32)), (np.zeros((1, 32, 3, 3)), np.zeros(1))]
    lap = -np.ones((3, 3)) / 8.0
    lap[1, 1] = 1.0
    P[0][0][0, 0] = lap
    P[0][1][0] = -theta
    for layer in (1, 2):
        P[layer][0][0, 0, 1, 1] = 1.0
    P[3][0][0, 0, 1, 1] = kappa
    return P
