"""k-space-only steps (SRBE_FLAG_KSPACE_ONLY) and the FP32 error split into its parts.

At fixed electrode charges and a given k-set, a k-space-only handle's ion forces are
compared with the oracle's Fourier force (Eq. (25)) plus the slab force, its b with
the oracle's Fourier and slab parts of b (Eq. (24) and the slab term), and a full
handle's forces minus the k-space-only ones with the oracle's real-space forces
(the gradients of Eq. (13)).  Tolerances per part: FP64 1e-11 relative (max-norm),
FP32 1e-5 relative RMS, as for the totals in test_gpu_step.py.
"""

import numpy as np
import pytest

from helpers import forces_from_soa, gpu_inputs, oracle_params, rel_inf, rel_rms
from oracle import ewald, sampler, srbe

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def pair():
    import paper_2509_24742_amd as srbe_amd
    from paper_2509_24742_amd import workloads as wl
    w = wl.tiny_slab()
    wp = dict(w["params"], kspace_tol=1e-16)
    full = srbe_amd.System(wp, w["ele_pos"], w["ele_side"], flags=srbe_amd.SRBE_FLAG_NO_CP)
    kso = srbe_amd.System(wp, w["ele_pos"], w["ele_side"],
                          flags=srbe_amd.SRBE_FLAG_NO_CP | srbe_amd.SRBE_FLAG_KSPACE_ONLY)
    yield dict(w=w, p=oracle_params(wp), full=full, kso=kso)
    full.close()
    kso.close()


def oracle_parts(p, ks, ion, q, ele, Q):
    ke = p.coulomb_k
    Fk = srbe.srbe_force_fourier(p, ks, ion, q, ele, Q)
    Mz = q @ ion[:, 2] + Q @ ele[:, 2]
    Fk[:, 2] -= ke * (4.0 * np.pi / p.V) * q * Mz
    bk = srbe.srbe_b_fourier(p, ks, ion, q, ele) - ke * (4.0 * np.pi / p.V) * ele[:, 2] * (q @ ion[:, 2])
    _, gii = ewald.real_space(p, "ii", ion, ion, q, same=True)
    _, gig = ewald.real_space(p, "ig", ion, ele, Q)
    Fr = -ke * q[:, None] * (gii + gig)
    return Fk, bk, Fr


@pytest.mark.parametrize("precision", [0, 1])
def test_kspace_and_real_space_parts(pair, precision):
    from paper_2509_24742_amd import binding
    w, p = pair["w"], pair["p"]
    ion, q, ele = np.asarray(w["ion_pos"]), np.asarray(w["ion_q"]), np.asarray(w["ele_pos"])
    ks, _ = sampler.draw_kset(p, 123, 0, 2)
    Q = np.random.default_rng(8).normal(size=len(ele)) * 0.05
    Q -= Q.mean()
    Fk_ref, bk_ref, Fr_ref = oracle_parts(p, ks, ion, q, ele, Q)
    off, xyz, qt, dp, sd = gpu_inputs([ion], [q], [w["dpsi"]], [0])
    kin = torch.tensor(ks.astype(np.int32).ravel(), device="cuda")
    qin = torch.tensor(Q, device="cuda")
    outs = {}
    for name in ("full", "kso"):
        outs[name] = pair[name].step(off, xyz, qt, dp, sd, 0, precision=precision, kset_in=kin, Q_in=qin)
        torch.cuda.synchronize()
        assert binding.srbe_sync_status(pair[name].h) == 0, binding.srbe_last_error(pair[name].h)
    Fk = forces_from_soa(outs["kso"]["F"], off, 0)
    Fr = forces_from_soa(outs["full"]["F"], off, 0) - Fk
    bk = outs["kso"]["b"].cpu().numpy()
    eFk, eFr, ebk = rel_rms(Fk, Fk_ref), rel_rms(Fr, Fr_ref), rel_rms(bk, bk_ref)
    print(f"precision {precision}: k-space force {eFk:.2e}, real-space force {eFr:.2e}, k-space b {ebk:.2e}",
          flush=True)
    if precision == 0:
        assert rel_inf(Fk, Fk_ref) < 1e-11 and rel_inf(Fr, Fr_ref) < 1e-11 and rel_inf(bk, bk_ref) < 1e-11
    else:
        assert eFk < 1e-5 and eFr < 1e-5 and ebk < 1e-5


def test_kspace_only_graph_advances_its_step(pair):
    # with no real-space pass and no energy output, the last launch still advances a
    # replayed graph's step counter: consecutive replays sample consecutive steps
    import paper_2509_24742_amd as srbe_amd
    w = pair["w"]
    off, xyz, qt, dp, sd = gpu_inputs([np.asarray(w["ion_pos"])], [np.asarray(w["ion_q"])], [w["dpsi"]], [5])
    Q = torch.zeros(pair["kso"].n_ele, dtype=torch.float64, device="cuda")
    out = pair["kso"].outputs(off, "cuda")
    gr = srbe_amd.srbe_graph_create(pair["kso"].h, srbe_amd.SRBE_FP32, off, xyz, qt, dp, sd, 10, out["Q"], out["F"],
                                    Q_in=Q, kset_out=out["kset"])
    try:
        got = []
        for _ in range(2):
            srbe_amd.srbe_graph_launch(gr)
            torch.cuda.synchronize()
            got.append(out["kset"].cpu().numpy().copy())
    finally:
        srbe_amd.srbe_graph_destroy(gr)
    p = pair["p"]
    for t, ks in enumerate(got):
        assert np.array_equal(ks.reshape(-1, 3), sampler.draw_kset(p, 5, 0, 10 + t)[0])
