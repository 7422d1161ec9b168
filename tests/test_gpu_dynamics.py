"""SRBE-driven dynamics: the short-range force field (srbe_ff_forces) and the captured
dynamics step (srbe_md_graph_create) through the C ABI.

* The force field on the paper-shaped cell (1,280 sites: three-site bonded cations,
  anions; walls placed to touch the nearest ions) against ``oracle.forcefield`` over all
  pairs: forces and the total energy to 1e-12 relative (FP64, same terms, other order).
* One replay of the dynamics graph on the tiny slab against the oracle's chain -- the
  SRBE step (``oracle.srbe``), plus the force field, then ``oracle.langevin`` -- to 1e-11
  relative in forces, positions and velocities (FP64).
* Replays of the graph equal the eager loop srbe_step -> srbe_ff_forces ->
  srbe_langevin_update bit for bit (both precisions).
"""

import numpy as np
import pytest

from helpers import gpu_inputs, oracle_params, oracle_solver, oracle_step, rel_inf

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

FF = dict(wca_eps=0.05, wca_sigma=0.3, wall_eps=0.2, wall_sigma=0.45, wall_zlo=0.8, wall_zhi=11.2, bond_k=500.0)


def _dev(a, dtype):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def test_ff_forces_match_oracle():
    import paper_2509_24742_amd as srbe_amd
    from oracle import forcefield
    from paper_2509_24742_amd import binding, workloads as wl
    w = wl.paper_cell()
    top = wl.paper_cell_topology()
    wp = dict(w["params"], kspace_tol=1e-16)
    sysm = srbe_amd.System(wp, w["ele_pos"], w["ele_side"], flags=srbe_amd.SRBE_FLAG_NO_CP)
    try:
        off, xyz, q, dp, sd = gpu_inputs([w["ion_pos"]], [w["ion_q"]], [w["dpsi"]], [7])
        n = len(w["ion_q"])
        sysm.step(off, xyz, q, dp, sd, 0, precision=0, Q_in=torch.zeros(sysm.n_ele, dtype=torch.float64,
                                                                          device="cuda"))
        F = torch.zeros(3 * n, dtype=torch.float64, device="cuda")
        e = torch.zeros(n, dtype=torch.float64, device="cuda")
        binding.srbe_ff_forces(sysm.h, 1, FF, _dev(top["mol"], torch.int32), _dev(top["bond"], torch.int32),
                               _dev(top["bond_r0"], torch.float64), F, e)
        torch.cuda.synchronize()
        got = F.cpu().numpy().reshape(3, n).T
        bonds = [(i, int(top["bond"][2 * i + u]), float(top["bond_r0"][2 * i + u])) for i in range(n) for u in range(2)
                 if top["bond"][2 * i + u] > i]
        ref = forcefield.forces(w["ion_pos"], top["mol"], bonds, FF, wp["Lx"], wp["Ly"])
        Eref = forcefield.energy(w["ion_pos"], top["mol"], bonds, FF, wp["Lx"], wp["Ly"])
        active = np.count_nonzero(np.any(ref != 0, axis=1))
        print(f"force field: {active} sites with a force, rel err {rel_inf(got, ref):.2e}, energy {Eref:.6f} "
              f"vs {float(e.sum()):.6f}", flush=True)
        assert active > 100
        assert rel_inf(got, ref) < 1e-12
        assert abs(float(e.sum()) - Eref) < 1e-12 * abs(Eref)
    finally:
        sysm.close()


def _tiny_md():
    from paper_2509_24742_amd import workloads as wl
    w = wl.tiny_slab()
    n = len(w["ion_q"])
    rng = np.random.default_rng(3)
    vel = rng.normal(size=(n, 3)) * 0.3
    mass = np.full(n, 40.0 / 96.485)
    ff = dict(FF, wall_zlo=0.1, wall_zhi=7.9)
    md = dict(ff=ff, gamma=0.5, beta=23.2, dt=0.002, zlo=0.3, zhi=7.7, noise_seed=99)
    top = dict(mol=np.arange(n, dtype=np.int32), bond=np.full(2 * n, -1, dtype=np.int32), bond_r0=np.zeros(2 * n))
    return w, vel, mass, md, top


@pytest.mark.parametrize("symplectic", [0, 1])
def test_md_graph_one_step_matches_oracle(symplectic):
    import paper_2509_24742_amd as srbe_amd
    from oracle import forcefield, langevin
    from paper_2509_24742_amd import binding
    w, vel, mass, md, top = _tiny_md()
    md = dict(md, symplectic=symplectic)
    wp = dict(w["params"], kspace_tol=1e-16)
    p = oracle_params(wp)
    sysm = srbe_amd.System(wp, w["ele_pos"], w["ele_side"])
    try:
        n = len(w["ion_q"])
        off, xyz, q, dp, sd = gpu_inputs([w["ion_pos"]], [w["ion_q"]], [w["dpsi"]], [2000])
        v = _dev(vel.T.ravel(), torch.float64)
        Q = torch.empty(sysm.n_ele, dtype=torch.float64, device="cuda")
        F = torch.empty(3 * n, dtype=torch.float64, device="cuda")
        gr = binding.srbe_md_graph_create(sysm.h, 0, off, xyz, v, q, _dev(mass, torch.float64),
                                          _dev(top["mol"], torch.int32), _dev(top["bond"], torch.int32),
                                          _dev(top["bond_r0"], torch.float64), dp, sd, 4, md, Q, F)
        binding.srbe_graph_launch(gr)
        torch.cuda.synchronize()
        assert binding.srbe_sync_status(sysm.h) == 0, binding.srbe_last_error(sysm.h)
        binding.srbe_graph_destroy(gr)
        ref = oracle_step(p, oracle_solver(p, w["ele_pos"]), 2000, 4, w["ion_pos"], w["ion_q"], w["ele_pos"],
                          w["ele_side"], w["dpsi"])
        Ft = ref["F"] + forcefield.forces(w["ion_pos"], top["mol"], [], md["ff"], wp["Lx"], wp["Ly"])
        r1, v1 = langevin.euler_maruyama(w["ion_pos"], vel, Ft, mass, md["gamma"], md["beta"], md["dt"], wp["Lx"],
                                         wp["Ly"], md["zlo"], md["zhi"], md["noise_seed"], 4,
                                         symplectic=bool(symplectic))
        got_F = F.cpu().numpy().reshape(3, n).T
        got_r = xyz.cpu().numpy().reshape(3, n).T
        got_v = v.cpu().numpy().reshape(3, n).T
        print(f"dynamics step: F {rel_inf(got_F, Ft):.2e}, r {rel_inf(got_r, r1):.2e}, v {rel_inf(got_v, v1):.2e}",
              flush=True)
        assert rel_inf(got_F, Ft) < 1e-11 and rel_inf(got_r, r1) < 1e-11 and rel_inf(got_v, v1) < 1e-11
        assert rel_inf(Q.cpu().numpy(), ref["Q"]) < 1e-11
    finally:
        sysm.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_md_graph_replays_equal_eager_loop(precision):
    import paper_2509_24742_amd as srbe_amd
    from paper_2509_24742_amd import binding
    w, vel, mass, md, top = _tiny_md()
    wp = dict(w["params"], kspace_tol=1e-16)
    sysm = srbe_amd.System(wp, w["ele_pos"], w["ele_side"])
    try:
        n = len(w["ion_q"])
        runs = []
        for mode in ("graph", "eager"):
            off, xyz, q, dp, sd = gpu_inputs([w["ion_pos"]], [w["ion_q"]], [w["dpsi"]], [2000])
            v = _dev(vel.T.ravel(), torch.float64)
            m = _dev(mass, torch.float64)
            mol, bond, r0 = (_dev(top["mol"], torch.int32), _dev(top["bond"], torch.int32),
                             _dev(top["bond_r0"], torch.float64))
            Q = torch.empty(sysm.n_ele, dtype=torch.float64, device="cuda")
            F = torch.empty(3 * n, dtype=torch.float64, device="cuda")
            if mode == "graph":
                gr = binding.srbe_md_graph_create(sysm.h, precision, off, xyz, v, q, m, mol, bond, r0, dp, sd, 10, md,
                                                  Q, F)
                for _ in range(3):
                    binding.srbe_graph_launch(gr)
                torch.cuda.synchronize()
                binding.srbe_graph_destroy(gr)
            else:
                ff = md["ff"]
                for step in (10, 11, 12):
                    sysm.step(off, xyz, q, dp, sd, step, precision=precision, out=dict(
                        Q=Q, F=F, b=None, psibar=torch.empty(1, dtype=torch.float64, device="cuda"),
                        E=torch.empty(1, dtype=torch.float64, device="cuda"), kset=None))
                    binding.srbe_ff_forces(sysm.h, 1, ff, mol, bond, r0, F)
                    binding.srbe_langevin_update(xyz, v, F, m, md["gamma"], md["beta"], md["dt"], wp["Lx"], wp["Ly"],
                                                 md["zlo"], md["zhi"], md["noise_seed"], step)
                torch.cuda.synchronize()
            assert binding.srbe_sync_status(sysm.h) == 0, binding.srbe_last_error(sysm.h)
            runs.append((xyz.cpu().numpy(), v.cpu().numpy(), F.cpu().numpy(), Q.cpu().numpy()))
        for a, b in zip(*runs):
            assert np.array_equal(a, b)
    finally:
        sysm.close()


def test_md_graph_keeps_its_buffers():
    # regression: the graph reads its topology, mass and state buffers at every replay.
    # Passed as temporaries, they must still be alive (the binding holds them) after
    # torch has allocated and filled other memory; the replays then equal those of a
    # graph whose buffers the caller keeps
    import paper_2509_24742_amd as srbe_amd
    from paper_2509_24742_amd import binding
    w, vel, mass, md, top = _tiny_md()
    wp = dict(w["params"], kspace_tol=1e-16)
    sysm = srbe_amd.System(wp, w["ele_pos"], w["ele_side"])
    try:
        n = len(w["ion_q"])
        runs = []
        for keep in (True, False):
            off, xyz, q, dp, sd = gpu_inputs([w["ion_pos"]], [w["ion_q"]], [w["dpsi"]], [2000])
            v = _dev(vel.T.ravel(), torch.float64)
            Q = torch.empty(sysm.n_ele, dtype=torch.float64, device="cuda")
            F = torch.empty(3 * n, dtype=torch.float64, device="cuda")
            held = (_dev(mass, torch.float64), _dev(top["mol"], torch.int32), _dev(top["bond"], torch.int32),
                    _dev(top["bond_r0"], torch.float64))
            if keep:
                gr = binding.srbe_md_graph_create(sysm.h, 1, off, xyz, v, q, *held, dp, sd, 10, md, Q, F)
            else:
                gr = binding.srbe_md_graph_create(sysm.h, 1, off, xyz, v, q, _dev(mass, torch.float64),
                                                  _dev(top["mol"], torch.int32), _dev(top["bond"], torch.int32),
                                                  _dev(top["bond_r0"], torch.float64), dp, sd, 10, md, Q, F)
                churn = [torch.full((4096,), 7, dtype=torch.int32, device="cuda") for _ in range(64)]
                del churn
            for _ in range(3):
                binding.srbe_graph_launch(gr)
            torch.cuda.synchronize()
            binding.srbe_graph_destroy(gr)
            assert binding.srbe_sync_status(sysm.h) == 0, binding.srbe_last_error(sysm.h)
            runs.append((xyz.cpu().numpy(), v.cpu().numpy(), F.cpu().numpy()))
        for a, b in zip(*runs):
            assert np.array_equal(a, b)
    finally:
        sysm.close()
