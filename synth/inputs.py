"""Workload descriptions and seeded input generators.

Workloads (atomic units):
  h_atom    H atom, Q2, box [-20,20]^3, 8^3 coarse cells, 2 levels in a
            2-bohr ball at the origin; 1 electron, 1 orbital; field-free,
            dt = 0.02, Krylov dimension 12, 100 steps.
  h2        H2, nuclei at z = +-0.7, Q3, box [-30,30]^3, 12^3 coarse cells,
            3 levels in 1.5-bohr balls around each nucleus; 2 electrons,
            2 orbitals (4 determinants); sin^2 pulse along z, 800 nm,
            E0 = 0.0534, 4 cycles, dt = 0.02, Krylov dimension 12.
  h2o       H2O geometry (O at the origin, H at (+-1.42994, 1.10718, 0)),
            Q3, box [-40,40]^3, 16^3 coarse cells, 4 levels within 6.5 bohr
            of O and 3 levels within 6.5 bohr of each H; CAS(10e, 8o);
            same pulse, 2 cycles.
  h2o_q1    the same molecule as the high-harmonic workload of Sec. IV:
            Q1, box [-64,64]^3 of 32^3 coarse cubes (edge 4 bohr), refined
            by Kelly's indicator of the nuclear potential (threshold 0.005,
            softening 0.05 bohr) down to edge 0.125 bohr (six cell sizes);
            CAS(10e, 8o); triangular 2-cycle pulse along x, 400 nm,
            8e14 W/cm^2 (E0 = 0.150982), dt = 0.01; velocity gauge (field
            values A(t)); exterior complex scaling at 0.3 rad beyond
            |x_d| = 44 (the refined cells end at 40, one 4-bohr layer inside).
  h2_batch  64 H2 instances, bond length ~ U[1,2], depth ~ {2,3,4},
            E0 ~ U[0.02, 0.06], drawn from default_rng(2301) in that order.

Nothing here evaluates the method; the pulse is an input field.
"""
import numpy as np

OMEGA_800NM = 0.0569542
OMEGA_400NM = 0.1139084
E0_1E14 = 0.0534
E0_8E14 = 0.150982


def _ball(center, radius, levels):
    return dict(center=tuple(float(v) for v in center), radius=float(radius), levels=int(levels))


def workload(name):
    """Geometry / molecule description of a named workload (plain dict)."""
    if name == "h_atom":
        return dict(name=name, lo=-20.0, hi=20.0, n_coarse=8, p=2,
                    balls=[_ball((0, 0, 0), 2.0, 2)],
                    nuclei=[(1.0, (0.0, 0.0, 0.0))], n_orb=1, n_alpha=1, n_beta=0,
                    dt=0.02, krylov=12, steps=100, E0=0.0, cycles=0)
    if name == "h2":
        R = 0.7
        return dict(name=name, lo=-30.0, hi=30.0, n_coarse=12, p=3,
                    balls=[_ball((0, 0, R), 1.5, 3), _ball((0, 0, -R), 1.5, 3)],
                    nuclei=[(1.0, (0.0, 0.0, R)), (1.0, (0.0, 0.0, -R))],
                    n_orb=2, n_alpha=1, n_beta=1, dt=0.02, krylov=12,
                    steps=22064, E0=E0_1E14, cycles=4)
    if name == "h2o":
        hx, hy = 1.42994, 1.10718
        return dict(name=name, lo=-40.0, hi=40.0, n_coarse=16, p=3,
                    balls=[_ball((0, 0, 0), 6.5, 4), _ball((hx, hy, 0), 6.5, 3),
                           _ball((-hx, hy, 0), 6.5, 3)],
                    nuclei=[(8.0, (0.0, 0.0, 0.0)), (1.0, (hx, hy, 0.0)), (1.0, (-hx, hy, 0.0))],
                    n_orb=8, n_alpha=5, n_beta=5, dt=0.02, krylov=12,
                    steps=11032, E0=E0_1E14, cycles=2)
    if name == "h2o_q1":
        hx, hy = 1.42994, 1.10718
        nuclei = [(8.0, (0.0, 0.0, 0.0)), (1.0, (hx, hy, 0.0)), (1.0, (-hx, hy, 0.0))]
        return dict(name=name, lo=-64.0, hi=64.0, n_coarse=32, p=1, balls=[],
                    kelly=dict(nuclei=nuclei, tol=0.005, soft=0.05, max_level=5),
                    nuclei=nuclei, n_orb=8, n_alpha=5, n_beta=5, dt=0.01, krylov=12,
                    E0=E0_8E14, cycles=2, omega=OMEGA_400NM, envelope="triangular", polarization=(1.0, 0.0, 0.0),
                    gauge="velocity", ecs=dict(theta=0.3, inner=(44.0, 44.0, 44.0)))
    raise KeyError(name)


def small_workload(name, seed=0):
    """Small meshes for parity cases (seconds for the oracle), several tiles
    and a ragged tail of cells; seeded ball placement."""
    rng = np.random.default_rng(seed)
    if name == "tiny_q2":
        return dict(name=name, lo=-6.0, hi=6.0, n_coarse=3, p=2,
                    balls=[_ball(rng.uniform(-1, 1, 3), 1.0, 1)],
                    nuclei=[(1.0, (0.0, 0.0, 0.0))], n_orb=1, n_alpha=1, n_beta=0)
    if name == "tiny_q3":
        c1 = rng.uniform(-1.5, 1.5, 3)
        return dict(name=name, lo=-8.0, hi=8.0, n_coarse=4, p=3,
                    balls=[_ball(c1, 1.2, 2), _ball(-c1, 0.8, 1)],
                    nuclei=[(1.0, tuple(c1 * 0.5)), (1.0, tuple(-c1 * 0.5))],
                    n_orb=2, n_alpha=1, n_beta=1)
    if name == "tiny_q1":
        return dict(name=name, lo=-5.0, hi=5.0, n_coarse=4, p=1,
                    balls=[_ball(rng.uniform(-0.5, 0.5, 3), 1.5, 2)],
                    nuclei=[(1.0, (0.3, -0.2, 0.1))], n_orb=2, n_alpha=1, n_beta=1)
    if name == "tiny_n8":   # eight orbitals: 64 real pair columns (column-blocked Poisson schedules)
        return dict(name=name, lo=-6.0, hi=6.0, n_coarse=3, p=2,
                    balls=[_ball(rng.uniform(-1, 1, 3), 1.0, 1)],
                    nuclei=[(3.0, (0.0, 0.0, 0.0))], n_orb=8, n_alpha=1, n_beta=1)
    if name == "tiny_n8_2a2b":   # eight orbitals, 2 alpha + 2 beta electrons: C(8,2)^2 = 784 determinants
        return dict(name=name, lo=-6.0, hi=6.0, n_coarse=3, p=2,
                    balls=[_ball(rng.uniform(-1, 1, 3), 1.0, 1)],
                    nuclei=[(4.0, (0.0, 0.0, 0.0))], n_orb=8, n_alpha=2, n_beta=2)
    if name == "small_n6":       # six orbitals, 3 alpha + 3 beta electrons: C(6,3)^2 = 400 determinants
        return dict(name=name, lo=-6.0, hi=6.0, n_coarse=3, p=2,
                    balls=[_ball((0.2, -0.3, 0.1), 1.5, 2)],
                    nuclei=[(6.0, (0.0, 0.0, 0.0))], n_orb=6, n_alpha=3, n_beta=3)
    if name == "h2_hmesh":  # H2 (nuclei at z = +-0.7, 2 orbitals) on the H-atom workload's Q2 mesh
        return dict(name=name, lo=-20.0, hi=20.0, n_coarse=8, p=2,
                    balls=[_ball((0, 0, 0), 2.0, 2)],
                    nuclei=[(1.0, (0.0, 0.0, 0.7)), (1.0, (0.0, 0.0, -0.7))], n_orb=2, n_alpha=1, n_beta=1)
    if name in ("kelly_q1", "kelly_q2"):  # H2 on a Kelly-refined mesh (no balls), field along x
        q1 = name == "kelly_q1"
        nuclei = [(1.0, (0.0, 0.0, 0.7)), (1.0, (0.0, 0.0, -0.7))]
        return dict(name=name, lo=-8.0, hi=8.0, n_coarse=4, p=1 if q1 else 2, balls=[],
                    kelly=dict(nuclei=nuclei, tol=0.01 if q1 else 0.005, soft=0.1, max_level=3),
                    nuclei=nuclei, n_orb=2, n_alpha=1, n_beta=1, polarization=(1.0, 0.0, 0.0))
    # exterior complex scaling cases: the refined block stays inside |x_d| < 4,
    # so every hanging node and master lies in unscaled cells; "ecs" gives the
    # angle and the inner half-widths (cell faces)
    if name == "ecs_q2":
        return dict(name=name, lo=-12.0, hi=12.0, n_coarse=6, p=2,
                    balls=[_ball(rng.uniform(-1, 1, 3), 1.0, 1)],
                    nuclei=[(1.0, (0.0, 0.0, 0.7)), (1.0, (0.0, 0.0, -0.7))], n_orb=2, n_alpha=1, n_beta=1,
                    polarization=(1.0, 0.0, 0.0), ecs=dict(theta=0.35, inner=(8.0, 8.0, 8.0)))
    if name == "ecs_q3":
        c1 = rng.uniform(-1.5, 1.5, 3)
        return dict(name=name, lo=-12.0, hi=12.0, n_coarse=6, p=3,
                    balls=[_ball(c1, 1.2, 1), _ball(-c1, 0.8, 1)],
                    nuclei=[(1.0, tuple(c1 * 0.5)), (1.0, tuple(-c1 * 0.5))], n_orb=2, n_alpha=1, n_beta=1,
                    polarization=(0.6, 0.0, 0.8), ecs=dict(theta=0.5, inner=(8.0, 8.0, 8.0)))
    if name == "ecs_n3":    # three orbitals, 9 determinants; y left unscaled
        return dict(name=name, lo=-12.0, hi=12.0, n_coarse=6, p=2,
                    balls=[_ball((0.2, -0.3, 0.1), 1.5, 1)],
                    nuclei=[(2.0, (0.0, 0.0, 0.0))], n_orb=3, n_alpha=2, n_beta=1,
                    polarization=(0.0, 0.0, 1.0), ecs=dict(theta=0.3, inner=(8.0, 12.0, 8.0)))
    if name == "kelly_ecs_q1":  # H2 on a Kelly mesh (refined within |x_d| < 16), scaled beyond 24
        nuclei = [(1.0, (0.0, 0.0, 0.7)), (1.0, (0.0, 0.0, -0.7))]
        return dict(name=name, lo=-32.0, hi=32.0, n_coarse=8, p=1, balls=[],
                    kelly=dict(nuclei=nuclei, tol=0.05, soft=0.1, max_level=4),
                    nuclei=nuclei, n_orb=2, n_alpha=1, n_beta=1, polarization=(1.0, 0.0, 0.0),
                    ecs=dict(theta=0.35, inner=(24.0, 24.0, 24.0)))
    if name == "small_n3":
        return dict(name=name, lo=-6.0, hi=6.0, n_coarse=3, p=2,
                    balls=[_ball((0.2, -0.3, 0.1), 1.5, 2)],
                    nuclei=[(2.0, (0.0, 0.0, 0.0))], n_orb=3, n_alpha=2, n_beta=1)
    raise KeyError(name)


def batch_instances(n=64, seed=2301):
    """H2 instances of the batched workload: (bond, depth, E0) per instance."""
    rng = np.random.default_rng(seed)
    R = rng.uniform(1.0, 2.0, n)
    depth = rng.integers(2, 5, n)
    E0 = rng.uniform(0.02, 0.06, n)
    out = []
    for i in range(n):
        h = R[i] / 2
        out.append(dict(name=f"h2_b{i}", lo=-30.0, hi=30.0, n_coarse=12, p=3,
                        balls=[_ball((0, 0, h), 1.5, depth[i]), _ball((0, 0, -h), 1.5, depth[i])],
                        nuclei=[(1.0, (0.0, 0.0, h)), (1.0, (0.0, 0.0, -h))],
                        n_orb=2, n_alpha=1, n_beta=1, dt=0.02, krylov=12, E0=float(E0[i]), cycles=4))
    return out


def pulse(t, E0, cycles, omega=OMEGA_800NM):
    """E(t) = E0 sin^2(pi t / Tp) sin(omega t) on [0, Tp], zero outside."""
    t = np.asarray(t, dtype=float)
    Tp = cycles * 2 * np.pi / omega if cycles else 1.0
    env = np.where((t >= 0) & (t <= Tp), np.sin(np.pi * t / Tp) ** 2, 0.0)
    return E0 * env * np.sin(omega * t)


def pulse_triangular(t, E0, omega=OMEGA_400NM):
    """E(t) = E0 f(t) sin(omega t) over two optical cycles, the envelope f
    rising linearly from 0 to 1 over the first cycle and falling back to 0
    over the second (the pulse of Sec. IV); zero outside."""
    t = np.asarray(t, dtype=float)
    ph = omega * t
    env = np.where((ph >= 0) & (ph <= 2 * np.pi), ph / (2 * np.pi),
                   np.where((ph > 2 * np.pi) & (ph <= 4 * np.pi), (4 * np.pi - ph) / (2 * np.pi), 0.0))
    return E0 * env * np.sin(ph)


def vector_potential_triangular(t, E0, omega=OMEGA_400NM):
    """A(t) = -int_0^t E of the triangular pulse, in closed form: with
    phi = omega t and c = E0 / (2 pi omega), int_0^t E = c (sin phi -
    phi cos phi) over the rising cycle and c ((phi - 4 pi) cos phi - sin phi)
    over the falling one, which ends at zero; zero outside the pulse."""
    t = np.asarray(t, dtype=float)
    ph = np.clip(omega * t, 0.0, 4 * np.pi)
    c = E0 / (2 * np.pi * omega)
    rise = np.sin(ph) - ph * np.cos(ph)
    fall = (ph - 4 * np.pi) * np.cos(ph) - np.sin(ph)
    return -c * np.where(ph <= 2 * np.pi, rise, fall)


def gaussian_orbitals(xyz, centers_exps, coeffs):
    """Columns sum_k coeffs[k, p] exp(-a_k |x - c_k|^2) at the points xyz."""
    cols = []
    for (c, a) in centers_exps:
        r2 = np.sum((xyz - np.asarray(c)[None, :]) ** 2, axis=1)
        cols.append(np.exp(-a * r2))
    B = np.stack(cols, axis=1)
    return B @ np.asarray(coeffs)


def random_orbitals(xyz, n, seed, n_gauss=6, spread=2.0):
    """Seeded smooth complex test functions (sums of Gaussians) at xyz."""
    rng = np.random.default_rng(seed)
    ce = [(rng.uniform(-spread, spread, 3), rng.uniform(0.3, 2.0)) for _ in range(n_gauss)]
    co = rng.standard_normal((n_gauss, n)) + 1j * rng.standard_normal((n_gauss, n))
    return gaussian_orbitals(xyz, ce, co)


def broad_orbitals(xyz, n, seed, length, n_gauss=6):
    """Seeded complex test functions spread over a region of the given
    length: Gaussians centred within +-length, of widths 0.7 to 1.4 length."""
    rng = np.random.default_rng(seed)
    ce = [(rng.uniform(-length, length, 3), rng.uniform(0.5, 2.0) / length ** 2) for _ in range(n_gauss)]
    co = rng.standard_normal((n_gauss, n)) + 1j * rng.standard_normal((n_gauss, n))
    return gaussian_orbitals(xyz, ce, co)


def random_ci(dim, seed):
    rng = np.random.default_rng(seed)
    C = rng.standard_normal(dim) + 1j * rng.standard_normal(dim)
    return C / np.linalg.norm(C)


def initial_guess(name, xyz):
    """Unnormalised initial orbital guesses at the points xyz."""
    if name in ("h_atom", "tiny_q2"):
        return gaussian_orbitals(xyz, [((0, 0, 0), 1.0)], np.array([[1.0]])).astype(complex)
    if name.startswith("h2") and name != "h2o":
        return None
    raise KeyError(name)


def h2_guess(xyz, half_bond):
    """sigma_g / sigma_u combinations of 1s-like Gaussians on the two nuclei."""
    ce = [((0, 0, half_bond), 0.8), ((0, 0, -half_bond), 0.8)]
    return gaussian_orbitals(xyz, ce, np.array([[1.0, 1.0], [1.0, -1.0]])).astype(complex)


def h2o_guess(xyz):
    """Eight Gaussian-type guesses: O 1s, 2s, 2px, 2py, 2pz and H 1s +- pair
    combinations (orthonormalised by the caller)."""
    hx, hy = 1.42994, 1.10718
    x, y, z = xyz[:, 0], xyz[:, 1], xyz[:, 2]
    r2 = x * x + y * y + z * z
    cols = [np.exp(-7.0 * r2), np.exp(-0.8 * r2) - 0.3 * np.exp(-7.0 * r2),
            x * np.exp(-0.9 * r2), y * np.exp(-0.9 * r2), z * np.exp(-0.9 * r2)]
    ha = np.exp(-0.9 * ((x - hx) ** 2 + (y - hy) ** 2 + z * z))
    hb = np.exp(-0.9 * ((x + hx) ** 2 + (y - hy) ** 2 + z * z))
    cols += [ha + hb, ha - hb, x * y * np.exp(-0.6 * r2)]
    return np.stack(cols, axis=1).astype(complex)


def h2_ci_guess():
    """CI start with every orbital occupied: (sqrt(0.99), 0, 0, -0.1)."""
    return np.array([np.sqrt(0.99), 0.0, 0.0, -0.1], dtype=complex)


def hf_ci(dim_alpha, dim_beta):
    """Lowest determinant (first alpha string x first beta string)."""
    C = np.zeros(dim_alpha * dim_beta, dtype=complex)
    C[0] = 1.0
    return C
