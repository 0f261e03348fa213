"""Helpers for the GPU tests: device copies of generator inputs."""
import numpy as np

import synth


def device_inputs(inp, torch):
    dev = torch.device("cuda:0")
    C = torch.from_numpy(inp.C).to(dev)
    V = torch.from_numpy(inp.V).to(dev)
    D = torch.from_numpy(inp.D).to(dev)
    return C, V, D


def run_build(plan, inp, torch, precision=0):
    C, V, D = device_inputs(inp, torch)
    K = torch.empty(plan.info["d_size"], dtype=torch.float64, device="cuda:0")
    Ex = torch.empty(plan.n_systems, dtype=torch.float64, device="cuda:0")
    plan.build_K(C, V, D, K, Ex, precision=precision)
    torch.cuda.synchronize()
    return K.cpu().numpy(), Ex.cpu().numpy()


def system_block(flat, layout, s):
    n = int(layout.sys_nbas[s])
    o = int(layout.sys_bas_off[s])
    return flat[o:o + n * n].reshape(n, n)


def relmax(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))
