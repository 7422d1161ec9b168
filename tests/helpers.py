"""Shared test plumbing: oracle set-up from a workload, and GPU inputs as torch tensors."""

import numpy as np

from oracle import cp, ewald, sampler, srbe


def oracle_params(wp, kspace_tol=1e-16):
    return ewald.Params(Lx=wp["Lx"], Ly=wp["Ly"], H=wp["H"], lam=wp["lam"], alpha=wp["alpha"], eta=wp["eta"],
                        rc=wp["rc"], coulomb_k=wp["coulomb_k"], M=int(wp["M"]), P=int(wp["P"]),
                        kspace_tol=kspace_tol)


def oracle_solver(p, ele_pos):
    return cp.Solver(ewald.electrode_matrix(p, ele_pos))


def oracle_step(p, solver, seed, step, ion_pos, ion_q, ele_pos, ele_side, dpsi, Q_fixed=None, kset=None):
    if kset is None:
        kset, _ = sampler.draw_kset(p, seed, 0, step)
    out = srbe.srbe_step(p, solver, kset, ion_pos, ion_q, ele_pos, ele_side, dpsi, Q_fixed=Q_fixed)
    out["kset"] = kset
    return out


def energy_scale(p, kset, ion_pos, ion_q, ele_side, dpsi, Q, b):
    """Sum of the magnitudes of the terms E* is assembled from (FP32 errors scale with it, not with |E*|)."""
    from oracle import ewald
    m, w = srbe._combined(p, kset)
    S1 = ewald.structure_factor(p, m, ion_pos, ion_q)
    phi, _ = ewald.real_space(p, "ii", ion_pos, ion_pos, ion_q, same=True)
    d = 0.5 * np.asarray(ele_side, dtype=np.float64)
    ke = p.coulomb_k
    terms = [0.5 * dpsi * d @ Q, 0.5 * b @ Q, 0.5 * ke * ion_q @ phi, 0.5 * ke * np.sum(w * np.abs(S1) ** 2),
             ke * p.alpha / np.sqrt(np.pi) * np.sum(ion_q ** 2), ke * 2 * np.pi / p.V * (ion_q @ ion_pos[:, 2]) ** 2]
    return float(np.sum(np.abs(terms)))


def gpu_inputs(ion_pos_list, ion_q_list, dpsi, seeds):
    """CSR offsets (host) and SoA device tensors for a list of replicas."""
    import torch
    sizes = [len(q) for q in ion_q_list]
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    pos = np.concatenate([np.asarray(p, dtype=np.float64).reshape(-1, 3) for p in ion_pos_list]) if sum(sizes) else np.zeros((0, 3))
    q = np.concatenate([np.asarray(x, dtype=np.float64) for x in ion_q_list]) if sum(sizes) else np.zeros(0)
    dev = torch.device("cuda")
    xyz = torch.tensor(np.ascontiguousarray(pos.T).ravel(), dtype=torch.float64, device=dev)
    qt = torch.tensor(q, dtype=torch.float64, device=dev)
    dp = torch.tensor(np.asarray(dpsi, dtype=np.float64), dtype=torch.float64, device=dev)
    sd = torch.tensor(np.asarray(seeds, dtype=np.uint64).view(np.int64), dtype=torch.int64, device=dev).view(torch.uint64)
    return off, xyz, qt, dp, sd


def forces_from_soa(F, off, r):
    """(n_r, 3) host forces of replica r from an SoA 3N device tensor."""
    N = int(off[-1])
    a = F.detach().cpu().numpy().reshape(3, N)
    return a[:, off[r]:off[r + 1]].T


def rel_inf(got, ref):
    got = np.asarray(got)
    ref = np.asarray(ref)
    return float(np.max(np.abs(got - ref)) / max(np.max(np.abs(ref)), 1e-300))


def rel_rms(got, ref):
    got = np.asarray(got)
    ref = np.asarray(ref)
    return float(np.linalg.norm(got - ref) / max(np.linalg.norm(ref), 1e-300))
