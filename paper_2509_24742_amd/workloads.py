"""Seeded synthetic electrode/electrolyte slabs.

This module only places particles and assigns charges (numpy, seeded); it holds
none of the method's arithmetic.  It feeds the same inputs to the GPU library and,
in the tests, to the CPU checker.

Units: nm, e, V.  Every workload is a dict with keys

  params   : dict(Lx, Ly, H, lam, alpha, eta, rc, coulomb_k, M, P)
  ion_pos  : float64 (N_ion, 3)      ion_q : float64 (N_ion,)
  ele_pos  : float64 (N_ele, 3)      ele_side : int8 (N_ele,) (-1 negative, +1 positive)
  dpsi     : float (V)

Placement recipes (the inputs stand in for the paper's MD snapshots of
graphene / coarse-grained ionic liquid, Sec. 4, which need a force field and an
equilibration run this project does not have):

* tiny slab: two 12x12 square walls (0.2 nm) at z = 0 and z = H = 8 nm in a
  2.4 x 2.4 nm cell; 100 + 100 ions of +-0.78 e placed by random sequential
  addition (RSA, 0.3 nm minimum separation, periodic in x and y) in
  z in [0.4, 7.6]; alpha = 3 /nm, eta = 1/19.79 nm, rc = 1.2 nm, M = 10, P = 100.
* paper-shaped cell: 3.4 x 3.7 x 12 nm; three honeycomb-topology layers of 360
  atoms per electrode (10 x 9 four-atom rectangular cells stretched to the box,
  AB-shifted, 0.335 nm apart); 320 rigid bent three-site cations
  (+0.1135, +0.2, +0.4665 e; 0.30 nm bonds at 120 degrees; random orientation)
  and 320 one-site anions (-0.78 e), RSA 0.3 nm in z in [1.07, H - 1.07];
  alpha = 3.5 /nm, eta = 0.0556 nm, rc = 1.2 nm, M = 13, P = 200.
* replica batch: R copies of the paper-shaped cell with placement seeds
  1100 + r and voltages drawn uniformly from [0, 4] V.
* per-step jitter: N(0, 0.01^2 nm^2) per axis and site; x, y wrap, z reflects
  back into the electrolyte interval.
* uneven batch: 32 systems (seed 4000), N log-uniform in [2e3, 2e5]; electrodes
  2 n^2 with n = round(sqrt(0.075 N)) on two n x n square walls; N_ion = N - 2 n^2
  made even (half +0.78 e, half -0.78 e); aspect Lz / Lx = lambda mu uniform in
  [3, 12] with lambda = 3; the electrolyte at 10 ions per nm^3 gives
  Lx = Ly = (3 N_ion / (10 lambda mu))^(1/3) and H = lambda mu Lx / 3; ions by
  RSA (0.3 nm) in z in [0.4, H - 0.4]; alpha = 3 /nm, eta = 1/19.79 nm,
  rc = 1.2 nm, M = ceil(lambda mu), P = round(100 sqrt(N / 1e4)), dpsi = 2 V.
* large slab: two n x n square walls (spacing Lx / n) at z = 0 and z = H in an
  Lx x Lx cell; n_ion ions of +-0.78 e (half each) by RSA (0.3 nm) in
  z in [0.4, H - 0.4]; alpha = 3 /nm, eta = 1/19.79 nm, rc = 1.2 nm.  The full
  size is 2 x 256 x 256 walls, 917,504 ions, 30 x 30 x 100 nm, M = 64, P = 500 or
  2000; smaller instances keep the density and the recipe.  Large placements use
  a batched RSA with the same acceptance rule (each candidate, in draw order, is
  kept if it is at least dmin from every site kept before it).
"""

import numpy as np

COULOMB_K = 1.43996454784  # e^2 / (4 pi eps0), in eV nm / e^2


def _rsa_accept(cand, placed, Lx, Ly, dmin):
    """True if every candidate site is at least dmin from every placed site (periodic in x, y)."""
    if placed is None or len(placed) == 0:
        return True
    d = cand[:, None, :] - placed[None, :, :]
    d[..., 0] -= Lx * np.round(d[..., 0] / Lx)
    d[..., 1] -= Ly * np.round(d[..., 1] / Ly)
    return bool(np.all(np.sum(d * d, axis=2) >= dmin * dmin))


def _rsa_sites(rng, n, Lx, Ly, zlo, zhi, dmin, max_tries=200000):
    placed = np.zeros((0, 3))
    tries = 0
    while len(placed) < n:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("random sequential addition did not converge")
        c = np.array([[rng.uniform(0, Lx), rng.uniform(0, Ly), rng.uniform(zlo, zhi)]])
        if _rsa_accept(c, placed, Lx, Ly, dmin):
            placed = np.vstack([placed, c])
    return placed


def _rsa_sites_batched(rng, n, Lx, Ly, zlo, zhi, dmin, batch=65536):
    """RSA of n sites, candidates drawn in batches and decided in draw order.

    A candidate is rejected if a site of an earlier batch lies within dmin
    (periodic in x and y; k-d tree), or if an earlier kept candidate of its own batch
    does (conflicting pairs of the batch visited in order of their later member).
    """
    from scipy.spatial import cKDTree
    box = (Lx, Ly, 4.0 * (zhi + dmin) + 1.0)  # z never wraps: the box is far taller than the sites
    placed = np.zeros((0, 3))
    while len(placed) < n:
        need = n - len(placed)
        m = int(min(batch, need * 1.1 + 64))
        cand = np.column_stack([rng.uniform(0, Lx, m), rng.uniform(0, Ly, m), rng.uniform(zlo, zhi, m)])
        cand[:, 0] %= Lx
        cand[:, 1] %= Ly
        if len(placed):
            d, _ = cKDTree(placed, boxsize=box).query(cand, k=1)
            cand = cand[d >= dmin]
        pairs = cKDTree(cand, boxsize=box).query_pairs(dmin, output_type="ndarray")
        keep = np.ones(len(cand), dtype=bool)
        if len(pairs):
            pairs = np.sort(pairs, axis=1)
            for i, j in pairs[np.argsort(pairs[:, 1], kind="stable")]:
                if keep[i]:
                    keep[j] = False
        placed = np.vstack([placed, cand[keep][:need]])
    return placed


def square_wall(n, a, z):
    g = (np.arange(n) + 0.5) * a
    X, Y = np.meshgrid(g, g, indexing="ij")
    return np.column_stack([X.ravel(), Y.ravel(), np.full(n * n, float(z))])


def honeycomb_layer(nx, ny, Lx, Ly, z, shift_frac=0.0):
    """4-atom rectangular honeycomb cells (fractions (0,0),(1/2,1/6),(1/2,1/2),(0,2/3)) stretched to Lx x Ly."""
    base = np.array([[0.0, 0.0], [0.5, 1.0 / 6.0], [0.5, 0.5], [0.0, 2.0 / 3.0]])
    cx, cy = Lx / nx, Ly / ny
    pts = []
    for i in range(nx):
        for j in range(ny):
            for b in base:
                x = (i + b[0]) * cx
                y = (j + b[1] + shift_frac) * cy
                pts.append([x % Lx, y % Ly, z])
    return np.array(pts)


def tiny_slab(seed=1000, dpsi=2.0):
    rng = np.random.default_rng(seed)
    Lx = Ly = 2.4
    H = 8.0
    ele = np.vstack([square_wall(12, 0.2, 0.0), square_wall(12, 0.2, H)])
    side = np.array([-1] * 144 + [1] * 144, dtype=np.int8)
    ion = _rsa_sites(rng, 200, Lx, Ly, 0.4, H - 0.4, 0.3)
    q = np.array([0.78] * 100 + [-0.78] * 100)
    params = dict(Lx=Lx, Ly=Ly, H=H, lam=3.0, alpha=3.0, eta=1.0 / 19.79, rc=1.2,
                  coulomb_k=COULOMB_K, M=10, P=100)
    return dict(params=params, ion_pos=ion, ion_q=q, ele_pos=ele, ele_side=side, dpsi=float(dpsi))


def large_slab(n_side=256, n_ion=917504, Lx=30.0, H=100.0, M=64, P=500, seed=1002, dpsi=2.0):
    """Square-wall slab at the large-system recipe; the defaults are the full size."""
    if n_ion % 2:
        raise ValueError("n_ion must be even")
    rng = np.random.default_rng(seed)
    a = Lx / n_side
    ele = np.vstack([square_wall(n_side, a, 0.0), square_wall(n_side, a, H)])
    side = np.array([-1] * n_side ** 2 + [1] * n_side ** 2, dtype=np.int8)
    ion = _rsa_sites_batched(rng, n_ion, Lx, Lx, 0.4, H - 0.4, 0.3)
    q = np.array([0.78] * (n_ion // 2) + [-0.78] * (n_ion // 2))
    params = dict(Lx=Lx, Ly=Lx, H=H, lam=3.0, alpha=3.0, eta=1.0 / 19.79, rc=1.2,
                  coulomb_k=COULOMB_K, M=M, P=P)
    return dict(params=params, ion_pos=ion, ion_q=q, ele_pos=ele, ele_side=side, dpsi=float(dpsi))


def uneven_batch(n_systems=32, seed=4000, place=True):
    """Systems of the uneven-batch recipe (a list of workload dicts, each with its own box).

    place: True places every system's ions; False none (ion_pos None: the sizes and
    boxes alone); a collection of indices, those systems only.  Each system's placement
    has its own generator (seed + 1 + index), so a system is the same whichever others
    are placed.
    """
    rng = np.random.default_rng(seed)
    N = np.exp(rng.uniform(np.log(2e3), np.log(2e5), n_systems)).astype(np.int64)
    aspect = rng.uniform(3.0, 12.0, n_systems)
    out = []
    for k in range(n_systems):
        n = int(round(np.sqrt(0.075 * N[k])))
        n_ion = int(N[k]) - 2 * n * n
        n_ion -= n_ion % 2
        Lx = (3.0 * n_ion / (10.0 * aspect[k])) ** (1.0 / 3.0)
        H = aspect[k] * Lx / 3.0
        a = Lx / n
        ele = np.vstack([square_wall(n, a, 0.0), square_wall(n, a, H)])
        side = np.array([-1] * n * n + [1] * n * n, dtype=np.int8)
        todo = place if isinstance(place, bool) else k in place
        ion = _rsa_sites_batched(np.random.default_rng(seed + 1 + k), n_ion, Lx, Lx, 0.4, H - 0.4, 0.3) if todo else None
        q = np.array([0.78] * (n_ion // 2) + [-0.78] * (n_ion // 2))
        params = dict(Lx=Lx, Ly=Lx, H=H, lam=3.0, alpha=3.0, eta=1.0 / 19.79, rc=1.2, coulomb_k=COULOMB_K,
                      M=int(np.ceil(aspect[k])), P=int(round(100.0 * np.sqrt(N[k] / 1e4))))
        out.append(dict(params=params, ion_pos=ion, ion_q=q, ele_pos=ele, ele_side=side, dpsi=2.0,
                        n_total=int(n_ion + 2 * n * n)))
    return out


CATION_Q = (0.1135, 0.2, 0.4665)
ANION_Q = -0.78


def _random_rotation(rng):
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    a, b, c, d = q
    return np.array([[a * a + b * b - c * c - d * d, 2 * (b * c - a * d), 2 * (b * d + a * c)],
                     [2 * (b * c + a * d), a * a - b * b + c * c - d * d, 2 * (c * d - a * b)],
                     [2 * (b * d - a * c), 2 * (c * d + a * b), a * a - b * b - c * c + d * d]])


def _cation_template():
    bond = 0.30
    ang = np.deg2rad(120.0)
    mid = np.zeros(3)
    e1 = np.array([bond, 0.0, 0.0])
    e2 = bond * np.array([np.cos(ang), np.sin(ang), 0.0])
    return np.array([e1, mid, e2])


def paper_cell(seed=1001, dpsi=2.0, n_pairs=320):
    rng = np.random.default_rng(seed)
    Lx, Ly, H = 3.4, 3.7, 12.0
    dz = 0.335
    layers = []
    for li, z in enumerate([0.0, dz, 2 * dz]):
        layers.append(honeycomb_layer(10, 9, Lx, Ly, z, shift_frac=(li % 2) / 3.0))
    for li, z in enumerate([H - 2 * dz, H - dz, H]):
        layers.append(honeycomb_layer(10, 9, Lx, Ly, z, shift_frac=(li % 2) / 3.0))
    ele = np.vstack(layers)
    side = np.array([-1] * 1080 + [1] * 1080, dtype=np.int8)
    zlo, zhi = 1.07, H - 1.07
    tmpl = _cation_template()
    placed = np.zeros((0, 3))
    cations = []
    tries = 0
    while len(cations) < n_pairs:
        tries += 1
        if tries > 500000:
            raise RuntimeError("cation placement did not converge")
        c = np.array([rng.uniform(0, Lx), rng.uniform(0, Ly), rng.uniform(zlo, zhi)])
        sites = c[None, :] + tmpl @ _random_rotation(rng).T
        if np.any(sites[:, 2] < zlo) or np.any(sites[:, 2] > zhi):
            continue
        sites[:, 0] %= Lx
        sites[:, 1] %= Ly
        if _rsa_accept(sites, placed, Lx, Ly, 0.3):
            placed = np.vstack([placed, sites])
            cations.append(sites)
    anions = []
    while len(anions) < n_pairs:
        tries += 1
        if tries > 1000000:
            raise RuntimeError("anion placement did not converge")
        c = np.array([[rng.uniform(0, Lx), rng.uniform(0, Ly), rng.uniform(zlo, zhi)]])
        if _rsa_accept(c, placed, Lx, Ly, 0.3):
            placed = np.vstack([placed, c])
            anions.append(c[0])
    ion = np.vstack([np.vstack(cations), np.array(anions)])
    q = np.concatenate([np.tile(CATION_Q, n_pairs), np.full(n_pairs, ANION_Q)])
    params = dict(Lx=Lx, Ly=Ly, H=H, lam=3.0, alpha=3.5, eta=0.0556, rc=1.2,
                  coulomb_k=COULOMB_K, M=13, P=200)
    return dict(params=params, ion_pos=ion, ion_q=q, ele_pos=ele, ele_side=side, dpsi=float(dpsi))


# masses (amu) of the coarse-grained ions of the paper's electrolyte: [BMIm]+ split over
# its three sites, [PF6]-
CATION_MASS = 139.22
ANION_MASS = 144.96


def paper_cell_topology(n_pairs=320):
    """Molecules, bonds and masses of paper_cell's sites (inputs of the dynamics).

    Sites are ordered as paper_cell places them: the three sites of every cation, then the
    anions.  Returns mol (molecule index per site), bond (two partner sites per site, -1
    none), bond_r0 (rest lengths: the template's 0.30 nm bonds and 0.52 nm between the end
    sites, which keeps the 120 degree angle) and mass (amu per site).
    """
    n = 4 * n_pairs
    mol = np.concatenate([np.repeat(np.arange(n_pairs), 3), n_pairs + np.arange(n_pairs)]).astype(np.int32)
    bond = np.full((n, 2), -1, dtype=np.int32)
    r0 = np.zeros((n, 2))
    tmpl = _cation_template()
    d_end = float(np.linalg.norm(tmpl[0] - tmpl[2]))
    for c in range(n_pairs):
        a, m, e = 3 * c, 3 * c + 1, 3 * c + 2
        bond[a] = (m, e)
        r0[a] = (0.30, d_end)
        bond[m] = (a, e)
        r0[m] = (0.30, 0.30)
        bond[e] = (m, a)
        r0[e] = (0.30, d_end)
    mass = np.concatenate([np.full(3 * n_pairs, CATION_MASS / 3.0), np.full(n_pairs, ANION_MASS)])
    return dict(mol=mol, bond=bond.ravel(), bond_r0=r0.ravel(), mass=mass)


def replica_batch(R=64, base_seed=1100, dpsi_seed=3000, n_pairs=320):
    """R paper-shaped cells sharing one electrode geometry; per-replica ions and voltage."""
    reps = [paper_cell(seed=base_seed + r, n_pairs=n_pairs) for r in range(R)]
    dpsi = np.random.default_rng(dpsi_seed).uniform(0.0, 4.0, size=R)
    out = dict(params=reps[0]["params"], ele_pos=reps[0]["ele_pos"], ele_side=reps[0]["ele_side"],
               ion_pos=[r["ion_pos"] for r in reps], ion_q=[r["ion_q"] for r in reps], dpsi=dpsi)
    return out


def jitter(pos, sigma, rng, Lx, Ly, zlo, zhi):
    """Gaussian per-axis displacement; x, y wrap into the cell, z reflects into [zlo, zhi]."""
    out = pos + rng.normal(scale=sigma, size=pos.shape)
    out[:, 0] %= Lx
    out[:, 1] %= Ly
    z = out[:, 2]
    z = np.where(z < zlo, 2 * zlo - z, z)
    z = np.where(z > zhi, 2 * zhi - z, z)
    out[:, 2] = z
    return out
