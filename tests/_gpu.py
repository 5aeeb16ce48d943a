"""Helpers that put an oracle problem on the GPU library (tests only)."""
import numpy as np

from paper_1705_06603_amd import _lib as dl

MODEL = {"interp": dl.MODEL_INTERP, "local": dl.MODEL_LOCAL}
REG = {"tv": dl.REG_SMOOTH_TV, "huber": dl.REG_HUBER}
BC = {"neumann": dl.BC_NEUMANN, "circular": dl.BC_CIRCULAR}


SOLVER = {"pg": dl.SOLVER_PG, "fista": dl.SOLVER_FISTA, "vmlmb": dl.SOLVER_VMLMB}


def params_of(problem, fft_size=0, local_solver="pg", independent=False):
    L = problem.layout
    ay, ax = L.ay, L.ax
    return dl.make_params(ay.M, ay.T, ay.p, ay.o, ay.G, 2 * ay.r + 1, model=MODEL[L.model],
                          reg=REG[problem.reg], bc=BC[problem.bc], positivity=problem.positivity,
                          fft_size=fft_size, lam=problem.lam, reg_param=problem.reg_param,
                          gamma=problem.gamma, rho=problem.rho, M_x=ax.M, T_x=ax.T, G_x=ax.G,
                          local_solver=SOLVER[local_solver], independent=independent,
                          layout=dl.LAYOUT_GRID if ay.kind == "grid" else dl.LAYOUT_PITCH)


def context_of(problem, fft_size=0, observe=True, local_solver="pg", independent=False):
    import torch
    ctx = dl.Context(params_of(problem, fft_size, local_solver, independent), problem.psfs)
    if observe:
        y = torch.tensor(problem.y, dtype=torch.float32, device="cuda").contiguous()
        W = torch.tensor(problem.W, dtype=torch.float32, device="cuda").contiguous()
        ctx.set_observation(y, W)
    return ctx


def to_dev(a):
    import torch
    return torch.tensor(np.asarray(a, dtype=np.float32), device="cuda").contiguous()


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))
