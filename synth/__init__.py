"""Seeded synthetic inputs for block-filtered EXC integration.

This module builds the *inputs* of the exchange-correlation integration: molecular geometries,
contracted cartesian Gaussian basis sets, atom-centred quadrature grids with Becke partition
weights, and a density matrix D = C C^T from orthonormalised random occupied orbitals.  Both the
CPU oracle and the HIP library consume what it produces; it contains none of the integration's own
arithmetic (no basis-on-grid evaluation, no density, no functional, no Fock contraction).

Units are atomic units throughout: positions in bohr, exponents in bohr^-2.  Geometry recipes are
stated in angstrom and converted with 1 A = 1/0.529177210903 bohr.

Recipes (one per workload; seeds: geometry 1000+k, basis 2000+k, orbitals 3000+k):

0  12 atoms (4 heavy, 8 light) uniform in an 8 A cube, min separation 1.0 A; grid 40 x 110;
   128-point blocks; 10 occupied orbitals; LDA.
1  100-step self-avoiding random walk of heavy atoms (1.4 A steps, nothing closer than 1.0 A), each
   capped by one H at 1.09 A in a random direction -> 200 atoms, 2000 AOs; grid 75 x 302; 128-point
   blocks; 400 occupied orbitals; PBE.
2  1000-atom globular cluster (500 heavy / 500 light, uniform in a sphere at 0.1 atoms/A^3, min
   separation 1.0 A); grid 75 x 302; 256-point blocks; 2000 occupied orbitals; PBE.
3  batch of 256 independent molecules: atom counts U{5..60} drawn from rng(4003); molecule j is
   built by the recipe of 0 with round(n/3) heavy atoms in a cube of side 8 A (n/12)^(1/3) (the
   atom density of 0), grid 50 x 194, round(N_AO/10) occupied orbitals, seeds (1000000+j,
   2000000+j, 3000000+j); the Becke partition keeps the atoms within 8 bohr as for 1, 2 and 4.
4  500-atom cluster by the recipe of 2; 1000 occupied orbitals.
Workloads 1, 2 and 4 keep, for each grid point, only the atoms within 8 bohr of its nearest atom in
the Becke partition (a partition of unity over that neighbour set); workload 0 uses all atoms.

Heavy atoms carry 3s2p1d shells (15 AOs), light atoms 2s1p (5 AOs).  Each shell has U{1..3}
primitives with exponents log-uniform in [0.1, 50] bohr^-2 (sorted descending) and contraction
coefficients U(0.1, 1) before normalisation.  The stored coefficients include the primitive
normalisation of the x^l component and a shell renormalisation to unit self-overlap; each cartesian
component (lx, ly, lz) is further scaled by sqrt((2l-1)!! / ((2lx-1)!! (2ly-1)!! (2lz-1)!!)) by the
consumer, which makes every AO unit-normalised.

Radial grid: Chebyshev quadrature of the second kind mapped by the Treutler-Ahlrichs M4 map
r = (xi/ln 2) (1+x)^0.6 ln(2/(1-x)), xi = 1 bohr.  Angular grid: spherical Fibonacci points with
equal weights 4 pi / N.  Partition: Becke 1988, three iterations, no size adjustment.

The density matrix is made from C ~ N(0,1) (N_AO x n_occ), orthonormalised in the metric of the
analytic overlap matrix S (Obara-Saika), so that tr(D S) = n_occ exactly.
"""
from __future__ import annotations

import ctypes
import hashlib
import math
import os
import subprocess
import sys
from dataclasses import dataclass, field

import numpy as np

GENERATOR_VERSION = "synth-v1"
BOHR_PER_ANGSTROM = 1.0 / 0.529177210903

HEAVY_SHELLS = (0, 0, 0, 1, 1, 2)   # 3s2p1d
LIGHT_SHELLS = (0, 0, 1)            # 2s1p

# cartesian component order within a shell: lexicographic (xx, xy, xz, yy, yz, zz)
CART_POWERS = {
    0: ((0, 0, 0),),
    1: ((1, 0, 0), (0, 1, 0), (0, 0, 1)),
    2: ((2, 0, 0), (1, 1, 0), (1, 0, 1), (0, 2, 0), (0, 1, 1), (0, 0, 2)),
}


def ncart(l: int) -> int:
    return (l + 1) * (l + 2) // 2


def _dfact(n: int) -> float:
    """(n)!! with (-1)!! = 1."""
    r = 1.0
    while n > 1:
        r *= n
        n -= 2
    return r


# --------------------------------------------------------------------------------------------
# containers
# --------------------------------------------------------------------------------------------
@dataclass
class Basis:
    shell_atom: np.ndarray      # int32 [n_shells]
    shell_l: np.ndarray         # int32 [n_shells]
    prim_ptr: np.ndarray        # int32 [n_shells+1]
    prim_exp: np.ndarray        # float64 [n_prim], bohr^-2
    prim_coef: np.ndarray       # float64 [n_prim], includes normalisation of the x^l component

    @property
    def n_shells(self) -> int:
        return int(self.shell_l.shape[0])

    @property
    def n_ao(self) -> int:
        return int(sum(ncart(int(l)) for l in self.shell_l))

    def ao_offsets(self) -> np.ndarray:
        """First AO (caller order) of each shell; AO order = shell order, components lexicographic."""
        n = np.array([ncart(int(l)) for l in self.shell_l], dtype=np.int64)
        return np.concatenate([[0], np.cumsum(n)[:-1]]).astype(np.int64)


@dataclass
class Grid:
    xyz: np.ndarray             # float64 [n_points, 3], bohr
    weight: np.ndarray          # float64 [n_points]
    point_atom: np.ndarray      # int32 [n_points], generating atom

    @property
    def n_points(self) -> int:
        return int(self.weight.shape[0])


@dataclass
class Problem:
    name: str
    atom_xyz: np.ndarray        # float64 [n_atoms, 3], bohr
    atom_heavy: np.ndarray      # bool [n_atoms]
    basis: Basis
    grid: Grid
    D: np.ndarray               # float64 [n_ao, n_ao], symmetric
    n_occ: int
    xc: str                     # "lda" or "pbe"
    grid_block: int = 128
    meta: dict = field(default_factory=dict)

    @property
    def n_atoms(self) -> int:
        return int(self.atom_xyz.shape[0])

    @property
    def n_ao(self) -> int:
        return self.basis.n_ao

    @property
    def n_points(self) -> int:
        return self.grid.n_points


# --------------------------------------------------------------------------------------------
# geometry
# --------------------------------------------------------------------------------------------
def _far_enough(pos, placed, min_sep):
    if not placed:
        return True
    d = np.linalg.norm(np.asarray(placed) - pos, axis=1)
    return bool(d.min() >= min_sep)


def cube_molecule(rng, n_heavy, n_light, box_A, min_sep_A=1.0):
    """Atoms uniform in a cube of side box_A with rejection below min_sep_A.  Returns bohr."""
    n = n_heavy + n_light
    placed = []
    tries = 0
    while len(placed) < n:
        p = rng.uniform(0.0, box_A, size=3)
        tries += 1
        if tries > 1000000:
            raise RuntimeError("cube_molecule: could not place atoms")
        if _far_enough(p, placed, min_sep_A):
            placed.append(p)
    heavy = np.zeros(n, dtype=bool)
    heavy[:n_heavy] = True
    return np.asarray(placed) * BOHR_PER_ANGSTROM, heavy


def _random_unit(rng):
    v = rng.normal(size=3)
    return v / np.linalg.norm(v)


def chain_molecule(rng, n_heavy, step_A=1.4, cap_A=1.09, min_sep_A=1.0):
    """Self-avoiding random walk of heavy atoms, each followed by one capping H.  Returns bohr."""
    placed = []
    heavy = []
    cur = np.zeros(3)
    for i in range(n_heavy):
        if i > 0:
            for _ in range(100000):
                cand = cur + step_A * _random_unit(rng)
                if _far_enough(cand, placed, min_sep_A):
                    break
            else:
                raise RuntimeError("chain_molecule: walk got stuck")
            cur = cand
        placed.append(cur.copy())
        heavy.append(True)
        for _ in range(100000):
            h = cur + cap_A * _random_unit(rng)
            if _far_enough(h, placed, min_sep_A):
                break
        else:
            raise RuntimeError("chain_molecule: could not cap atom")
        placed.append(h)
        heavy.append(False)
    return np.asarray(placed) * BOHR_PER_ANGSTROM, np.asarray(heavy, dtype=bool)


def sphere_cluster(rng, n_heavy, n_light, density_A3=0.1, min_sep_A=1.0):
    """Atoms uniform in a sphere at the given number density; heavy and light interleaved."""
    n = n_heavy + n_light
    R = (3.0 * n / (4.0 * math.pi * density_A3)) ** (1.0 / 3.0)
    placed = []
    tries = 0
    while len(placed) < n:
        p = rng.uniform(-R, R, size=3)
        tries += 1
        if tries > 50000000:
            raise RuntimeError("sphere_cluster: could not place atoms")
        if p @ p > R * R:
            continue
        if _far_enough(p, placed, min_sep_A):
            placed.append(p)
    heavy = np.zeros(n, dtype=bool)
    heavy[0::2][: n_heavy] = True
    if heavy.sum() != n_heavy:
        heavy[:] = False
        heavy[:n_heavy] = True
    return np.asarray(placed) * BOHR_PER_ANGSTROM, heavy


# --------------------------------------------------------------------------------------------
# basis
# --------------------------------------------------------------------------------------------
def _prim_norm(alpha, l):
    """Normalisation of x^l exp(-alpha r^2)."""
    return (2.0 * alpha / math.pi) ** 0.75 * (4.0 * alpha) ** (l / 2.0) / math.sqrt(_dfact(2 * l - 1))


def make_basis(rng, atom_heavy, exp_range=(0.1, 50.0), nprim_range=(1, 3)) -> Basis:
    shell_atom, shell_l, ptr, exps, coefs = [], [], [0], [], []
    lo, hi = math.log(exp_range[0]), math.log(exp_range[1])
    for a, hv in enumerate(atom_heavy):
        for l in (HEAVY_SHELLS if hv else LIGHT_SHELLS):
            k = int(rng.integers(nprim_range[0], nprim_range[1] + 1))
            al = np.sort(np.exp(rng.uniform(lo, hi, size=k)))[::-1]
            c = rng.uniform(0.1, 1.0, size=k)
            c = c * np.array([_prim_norm(x, l) for x in al])
            # renormalise the shell: <x^l g | x^l g> = 1
            s = 0.0
            for i in range(k):
                for j in range(k):
                    p = al[i] + al[j]
                    s += c[i] * c[j] * _dfact(2 * l - 1) / (2.0 * p) ** l * (math.pi / p) ** 1.5
            c = c / math.sqrt(s)
            shell_atom.append(a)
            shell_l.append(l)
            exps.extend(al.tolist())
            coefs.extend(c.tolist())
            ptr.append(len(exps))
    return Basis(np.asarray(shell_atom, np.int32), np.asarray(shell_l, np.int32),
                 np.asarray(ptr, np.int32), np.asarray(exps, np.float64), np.asarray(coefs, np.float64))


# --------------------------------------------------------------------------------------------
# grid
# --------------------------------------------------------------------------------------------
def radial_grid(n, xi=1.0):
    """Chebyshev (2nd kind) nodes on (-1,1) mapped to (0, inf) by the Treutler-Ahlrichs M4 map.

    Returns (r, w) with sum_i w_i g(r_i) ~= int_0^inf g(r) r^2 dr."""
    i = np.arange(1, n + 1, dtype=np.float64)
    t = i * math.pi / (n + 1)
    x = np.cos(t)
    wx = math.pi / (n + 1) * np.sin(t)          # = pi/(n+1) sin^2(t) / sqrt(1-x^2)
    a = 0.6
    L = np.log(2.0 / (1.0 - x))
    r = xi / math.log(2.0) * (1.0 + x) ** a * L
    drdx = xi / math.log(2.0) * (a * (1.0 + x) ** (a - 1.0) * L + (1.0 + x) ** a / (1.0 - x))
    return r, wx * r * r * drdx


def fibonacci_sphere(n):
    """Spherical Fibonacci points (unit vectors) with equal weights 4 pi / n."""
    k = np.arange(n, dtype=np.float64)
    z = 1.0 - (2.0 * k + 1.0) / n
    rho = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    phi = k * math.pi * (3.0 - math.sqrt(5.0))
    u = np.stack([rho * np.cos(phi), rho * np.sin(phi), z], axis=1)
    return u, np.full(n, 4.0 * math.pi / n)


_BECKE_LIB = None


def _becke_lib():
    global _BECKE_LIB
    if _BECKE_LIB is not None:
        return _BECKE_LIB
    here = os.path.dirname(os.path.abspath(__file__))
    src = os.path.join(here, "becke.c")
    so = os.path.join(here, "_becke.so")
    if not os.path.exists(so) or os.path.getmtime(so) < os.path.getmtime(src):
        build_becke()
    lib = ctypes.CDLL(so)
    lib.becke_fractions.restype = ctypes.c_int
    lib.becke_fractions.argtypes = [ctypes.c_int32, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                    ctypes.c_void_p, ctypes.c_double, ctypes.c_void_p]
    _BECKE_LIB = lib
    return lib


def build_becke():
    """Compile the Becke partition helper (plain C, OpenMP) next to this file."""
    here = os.path.dirname(os.path.abspath(__file__))
    src = os.path.join(here, "becke.c")
    so = os.path.join(here, "_becke.so")
    tmp = so + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", tmp, src, "-lm"])
    os.replace(tmp, so)
    return so


def becke_fractions(atom_xyz, pts, pt_atom, cutoff=0.0):
    lib = _becke_lib()
    atom_xyz = np.ascontiguousarray(atom_xyz, np.float64)
    pts = np.ascontiguousarray(pts, np.float64)
    pt_atom = np.ascontiguousarray(pt_atom, np.int32)
    out = np.empty(pts.shape[0], np.float64)
    rc = lib.becke_fractions(atom_xyz.shape[0], atom_xyz.ctypes.data, pts.shape[0], pts.ctypes.data,
                             pt_atom.ctypes.data, float(cutoff), out.ctypes.data)
    if rc != 0:
        raise RuntimeError("becke_fractions failed (%d)" % rc)
    return out


def make_grid(atom_xyz, n_rad, n_ang, becke_cutoff=0.0) -> Grid:
    """Atom-centred product grid; points are generated atom-major, radial-major, angular-minor."""
    r, wr = radial_grid(n_rad)
    u, wa = fibonacci_sphere(n_ang)
    n_atoms = atom_xyz.shape[0]
    local = (r[:, None, None] * u[None, :, :]).reshape(-1, 3)
    wloc = (wr[:, None] * wa[None, :]).reshape(-1)
    pts = (atom_xyz[:, None, :] + local[None, :, :]).reshape(-1, 3)
    pt_atom = np.repeat(np.arange(n_atoms, dtype=np.int32), local.shape[0])
    frac = becke_fractions(atom_xyz, pts, pt_atom, becke_cutoff) if n_atoms > 1 else np.ones(len(pts))
    w = np.tile(wloc, n_atoms) * frac
    return Grid(pts, w, pt_atom)


# --------------------------------------------------------------------------------------------
# analytic overlap (Obara-Saika) and the density matrix
# --------------------------------------------------------------------------------------------
def _os_1d(la, lb, PA, PB, inv2p):
    """1D Obara-Saika overlap table s[i][j] / s00, i<=la, j<=lb, vectorised over the last axis."""
    s = {}
    one = np.ones_like(PA)
    s[(0, 0)] = one
    for i in range(la + 1):
        for j in range(lb + 1):
            if (i, j) == (0, 0):
                continue
            if i > 0:
                v = PA * s[(i - 1, j)]
                if i > 1:
                    v = v + (i - 1) * inv2p * s[(i - 2, j)]
                if j > 0:
                    v = v + j * inv2p * s[(i - 1, j - 1)]
            else:
                v = PB * s[(i, j - 1)]
                if j > 1:
                    v = v + (j - 1) * inv2p * s[(i, j - 2)]
            s[(i, j)] = v
    return s


def overlap_matrix(basis: Basis, atom_xyz) -> np.ndarray:
    """Analytic overlap S_{mu nu} = <chi_mu | chi_nu> of the unit-normalised cartesian AOs."""
    nsh = basis.n_shells
    off = basis.ao_offsets()
    nao = basis.n_ao
    S = np.zeros((nao, nao))
    ls = basis.shell_l
    ctr = atom_xyz[basis.shell_atom]
    nrel = {l: np.array([math.sqrt(_dfact(2 * l - 1) / (_dfact(2 * a - 1) * _dfact(2 * b - 1) * _dfact(2 * c - 1)))
                         for (a, b, c) in CART_POWERS[l]]) for l in CART_POWERS}
    # primitive lists padded to 3 per shell
    maxk = int(np.max(np.diff(basis.prim_ptr)))
    pe = np.zeros((nsh, maxk))
    pc = np.zeros((nsh, maxk))
    for s in range(nsh):
        a0, a1 = basis.prim_ptr[s], basis.prim_ptr[s + 1]
        pe[s, : a1 - a0] = basis.prim_exp[a0:a1]
        pc[s, : a1 - a0] = basis.prim_coef[a0:a1]
    for la in range(3):
        sa = np.nonzero(ls == la)[0]
        for lb in range(3):
            sb = np.nonzero(ls == lb)[0]
            if len(sa) == 0 or len(sb) == 0:
                continue
            I, J = np.meshgrid(sa, sb, indexing="ij")
            I = I.ravel()
            J = J.ravel()
            A = ctr[I]
            B = ctr[J]
            AB2 = np.sum((A - B) ** 2, axis=1)
            block = np.zeros((len(I), ncart(la), ncart(lb)))
            for ka in range(maxk):
                for kb in range(maxk):
                    a = pe[I, ka]
                    b = pe[J, kb]
                    m = (a > 0) & (b > 0)
                    if not np.any(m):
                        continue
                    a = np.where(m, a, 1.0)
                    b = np.where(m, b, 1.0)
                    p = a + b
                    P = (a[:, None] * A + b[:, None] * B) / p[:, None]
                    s00 = (math.pi / p) ** 1.5 * np.exp(-a * b / p * AB2)
                    coef = np.where(m, pc[I, ka] * pc[J, kb], 0.0) * s00
                    inv2p = 0.5 / p
                    tabs = [_os_1d(la, lb, P[:, d] - A[:, d], P[:, d] - B[:, d], inv2p) for d in range(3)]
                    for u, (ax, ay, az) in enumerate(CART_POWERS[la]):
                        for v, (bx, by, bz) in enumerate(CART_POWERS[lb]):
                            block[:, u, v] += coef * tabs[0][(ax, bx)] * tabs[1][(ay, by)] * tabs[2][(az, bz)]
            block *= nrel[la][None, :, None] * nrel[lb][None, None, :]
            na, nb = ncart(la), ncart(lb)
            rows = off[I][:, None, None] + np.arange(na)[None, :, None]
            cols = off[J][:, None, None] + np.arange(nb)[None, None, :]
            S[np.broadcast_to(rows, block.shape), np.broadcast_to(cols, block.shape)] = block
    return 0.5 * (S + S.T)


def make_density(rng, S, n_occ):
    """D = C C^T with C ~ N(0,1) orthonormalised so that C^T S C = 1."""
    nao = S.shape[0]
    C = rng.normal(size=(nao, n_occ))
    M = C.T @ S @ C
    L = np.linalg.cholesky(0.5 * (M + M.T))
    C = np.linalg.solve(L, C.T).T          # C L^{-T}
    D = C @ C.T
    return 0.5 * (D + D.T)


# --------------------------------------------------------------------------------------------
# workloads
# --------------------------------------------------------------------------------------------
RECIPES = {
    0: dict(kind="cube", n_heavy=4, n_light=8, box_A=8.0, n_rad=40, n_ang=110, G=128, n_occ=10, xc="lda"),
    1: dict(kind="chain", n_heavy=100, n_rad=75, n_ang=302, G=128, n_occ=400, xc="pbe", becke_cutoff=8.0),
    2: dict(kind="sphere", n_heavy=500, n_light=500, n_rad=75, n_ang=302, G=256, n_occ=2000, xc="pbe",
            becke_cutoff=8.0),
    4: dict(kind="sphere", n_heavy=250, n_light=250, n_rad=75, n_ang=302, G=256, n_occ=1000, xc="pbe",
            becke_cutoff=8.0),
}


def _cache_dir():
    d = os.environ.get("KLDI_SYNTH_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "kldi_synth"))
    os.makedirs(d, exist_ok=True)
    return d


def build_problem(recipe: dict, seeds=(1000, 2000, 3000), name="custom") -> Problem:
    """Build a problem from a recipe dict (see RECIPES) with explicit seeds (geometry, basis, orbitals)."""
    g_rng = np.random.default_rng(seeds[0])
    kind = recipe["kind"]
    if kind == "cube":
        xyz, heavy = cube_molecule(g_rng, recipe["n_heavy"], recipe["n_light"], recipe["box_A"],
                                   recipe.get("min_sep_A", 1.0))
    elif kind == "chain":
        xyz, heavy = chain_molecule(g_rng, recipe["n_heavy"])
    elif kind == "sphere":
        xyz, heavy = sphere_cluster(g_rng, recipe["n_heavy"], recipe["n_light"])
    elif kind == "explicit":
        xyz = np.asarray(recipe["atoms_bohr"], np.float64).reshape(-1, 3)
        heavy = np.asarray(recipe["heavy"], bool)
    else:
        raise ValueError(kind)
    basis = make_basis(np.random.default_rng(seeds[1]), heavy,
                       exp_range=recipe.get("exp_range", (0.1, 50.0)),
                       nprim_range=recipe.get("nprim_range", (1, 3)))
    grid = make_grid(xyz, recipe["n_rad"], recipe["n_ang"], recipe.get("becke_cutoff", 0.0))
    S = overlap_matrix(basis, xyz)
    D = make_density(np.random.default_rng(seeds[2]), S, recipe["n_occ"])
    return Problem(name=name, atom_xyz=xyz, atom_heavy=heavy, basis=basis, grid=grid, D=D,
                   n_occ=int(recipe["n_occ"]), xc=recipe["xc"], grid_block=int(recipe.get("G", 128)),
                   meta=dict(recipe=dict(recipe), seeds=list(seeds), generator=GENERATOR_VERSION))


def _save(p: Problem, path):
    tmp = path + ".tmp%d.npz" % os.getpid()
    np.savez(tmp, atom_xyz=p.atom_xyz, atom_heavy=p.atom_heavy, shell_atom=p.basis.shell_atom,
             shell_l=p.basis.shell_l, prim_ptr=p.basis.prim_ptr, prim_exp=p.basis.prim_exp,
             prim_coef=p.basis.prim_coef, gxyz=p.grid.xyz, gw=p.grid.weight, gatom=p.grid.point_atom,
             D=p.D, n_occ=p.n_occ, xc=p.xc, G=p.grid_block, name=p.name)
    os.replace(tmp, path)


def _load(path, meta) -> Problem:
    z = np.load(path, allow_pickle=False)
    basis = Basis(z["shell_atom"], z["shell_l"], z["prim_ptr"], z["prim_exp"], z["prim_coef"])
    grid = Grid(z["gxyz"], z["gw"], z["gatom"])
    return Problem(name=str(z["name"]), atom_xyz=z["atom_xyz"], atom_heavy=z["atom_heavy"], basis=basis,
                   grid=grid, D=z["D"], n_occ=int(z["n_occ"]), xc=str(z["xc"]), grid_block=int(z["G"]),
                   meta=meta)


def make_problem(k: int, cache=True) -> Problem:
    """Workload k of the recipe table, built from its fixed seeds (cached as .npz)."""
    recipe = RECIPES[k]
    seeds = (1000 + k, 2000 + k, 3000 + k)
    meta = dict(recipe=dict(recipe), seeds=list(seeds), generator=GENERATOR_VERSION)
    key = hashlib.sha1(repr((GENERATOR_VERSION, sorted(recipe.items()), seeds)).encode()).hexdigest()[:16]
    path = os.path.join(_cache_dir(), "cfg%d_%s.npz" % (k, key))
    if cache and os.path.exists(path):
        return _load(path, meta)
    p = build_problem(recipe, seeds, name="cfg%d" % k)
    if cache:
        _save(p, path)
    return p


def subset_problem(k: int, n_sub=200, G=128, cache=True) -> Problem:
    """The n_sub atoms of cluster workload k nearest its centroid, as a problem of their own.

    Geometry and basis are those of workload k (same seeds): the selected atoms keep their positions
    and shells, in their order in the cluster.  The grid (the recipe's radial x angular points, Becke
    partition over the subset) and D (orbital seed 3100+k, round(N_AO/5) occupied orbitals, the
    occupied-orbital ratio of the recipe) are built for the subset alone.  Ties in the distance are
    broken by atom index.
    """
    recipe = RECIPES[k]
    if recipe["kind"] != "sphere":
        raise ValueError("subset_problem: workload %d is not a cluster" % k)
    seeds = (1000 + k, 2000 + k, 3100 + k)
    meta = dict(recipe=dict(recipe), seeds=list(seeds), generator=GENERATOR_VERSION,
                subset=dict(of=k, n_atoms=n_sub, rule="nearest to the centroid"))
    key = hashlib.sha1(repr((GENERATOR_VERSION, sorted(recipe.items()), seeds, n_sub, G)).encode()).hexdigest()[:16]
    path = os.path.join(_cache_dir(), "cfg%dsub%d_%s.npz" % (k, n_sub, key))
    if cache and os.path.exists(path):
        return _load(path, meta)
    xyz, heavy = sphere_cluster(np.random.default_rng(seeds[0]), recipe["n_heavy"], recipe["n_light"])
    full = make_basis(np.random.default_rng(seeds[1]), heavy)
    d = np.linalg.norm(xyz - xyz.mean(axis=0), axis=1)
    sel = np.sort(np.lexsort((np.arange(len(d)), d))[:n_sub])
    new_index = -np.ones(len(xyz), np.int64)
    new_index[sel] = np.arange(n_sub)
    keep = np.flatnonzero(new_index[full.shell_atom] >= 0)
    ptr, exps, coefs = [0], [], []
    for s in keep:
        a0, a1 = full.prim_ptr[s], full.prim_ptr[s + 1]
        exps.extend(full.prim_exp[a0:a1].tolist())
        coefs.extend(full.prim_coef[a0:a1].tolist())
        ptr.append(len(exps))
    basis = Basis(new_index[full.shell_atom[keep]].astype(np.int32), full.shell_l[keep].astype(np.int32),
                  np.asarray(ptr, np.int32), np.asarray(exps, np.float64), np.asarray(coefs, np.float64))
    sxyz = xyz[sel]
    grid = make_grid(sxyz, recipe["n_rad"], recipe["n_ang"], recipe.get("becke_cutoff", 0.0))
    n_occ = int(round(basis.n_ao / 5.0))
    D = make_density(np.random.default_rng(seeds[2]), overlap_matrix(basis, sxyz), n_occ)
    p = Problem(name="cfg%dsub%d" % (k, n_sub), atom_xyz=sxyz, atom_heavy=heavy[sel], basis=basis, grid=grid,
                D=D, n_occ=n_occ, xc=recipe["xc"], grid_block=G, meta=meta)
    if cache:
        _save(p, path)
    return p


def tiny_problem(n_atoms=3, n_rad=12, n_ang=26, n_occ=3, xc="lda", seed=7, heavy=None, box_A=3.0, G=128):
    """Small seeded problem for unit tests (ragged AO count and grid length by construction)."""
    n_heavy = (n_atoms + 1) // 2 if heavy is None else heavy
    recipe = dict(kind="cube", n_heavy=n_heavy, n_light=n_atoms - n_heavy, box_A=box_A, n_rad=n_rad,
                  n_ang=n_ang, G=G, n_occ=n_occ, xc=xc, min_sep_A=0.9)
    return build_problem(recipe, (seed, seed + 1, seed + 2), name="tiny%d" % seed)


# --------------------------------------------------------------------------------------------
# batches of independent molecules
# --------------------------------------------------------------------------------------------
BATCH_RECIPE = dict(n_mol=256, atoms=(5, 60), n_rad=50, n_ang=194, G=128, becke_cutoff=8.0, seed=4003)


def batch_member(n_atoms, j, n_rad=50, n_ang=194, xc="lda", becke_cutoff=8.0):
    """Molecule j of a batch: the recipe of workload 0 scaled to n_atoms at the same atom density."""
    n_heavy = int(round(n_atoms / 3.0))
    box = 8.0 * (n_atoms / 12.0) ** (1.0 / 3.0)
    g_rng = np.random.default_rng(1000000 + j)
    xyz, heavy = cube_molecule(g_rng, n_heavy, n_atoms - n_heavy, box)
    basis = make_basis(np.random.default_rng(2000000 + j), heavy)
    grid = make_grid(xyz, n_rad, n_ang, becke_cutoff)
    S = overlap_matrix(basis, xyz)
    n_occ = max(1, int(round(basis.n_ao / 10.0)))
    D = make_density(np.random.default_rng(3000000 + j), S, n_occ)
    return Problem(name="mol%d" % j, atom_xyz=xyz, atom_heavy=heavy, basis=basis, grid=grid, D=D, n_occ=n_occ,
                   xc=xc, grid_block=128, meta=_member_meta(n_atoms, j, n_rad, n_ang, becke_cutoff))


def _member_meta(n_atoms, j, n_rad, n_ang, becke_cutoff):
    n_heavy = int(round(n_atoms / 3.0))
    box = 8.0 * (n_atoms / 12.0) ** (1.0 / 3.0)
    return dict(recipe=dict(kind="cube", n_heavy=n_heavy, n_light=n_atoms - n_heavy, box_A=box, n_rad=n_rad,
                            n_ang=n_ang, becke_cutoff=becke_cutoff),
                seeds=[1000000 + j, 2000000 + j, 3000000 + j], generator=GENERATOR_VERSION)


def batch_sizes(n_mol=256, atoms=(5, 60), seed=4003):
    """Atom counts of the molecules of a batch, U{atoms[0]..atoms[1]}."""
    return np.random.default_rng(seed).integers(atoms[0], atoms[1] + 1, size=n_mol)


def make_batch(n_mol=None, atoms=None, n_rad=None, n_ang=None, xc="lda", cache=True):
    """The molecules of the batching workload (defaults: BATCH_RECIPE); the first n_mol of them if
    n_mol is smaller than 256 (sizes always come from the same draw)."""
    r = dict(BATCH_RECIPE)
    for k, v in (("n_mol", n_mol), ("atoms", atoms), ("n_rad", n_rad), ("n_ang", n_ang)):
        if v is not None:
            r[k] = v
    sizes = batch_sizes(max(r["n_mol"], 1), r["atoms"], r["seed"])[: r["n_mol"]]
    out = []
    for j, n in enumerate(sizes):
        key = hashlib.sha1(repr((GENERATOR_VERSION, int(n), j, r["n_rad"], r["n_ang"], r["becke_cutoff"])).encode()
                           ).hexdigest()[:16]
        path = os.path.join(_cache_dir(), "batch_%s.npz" % key)
        if cache and os.path.exists(path):
            p = _load(path, _member_meta(int(n), j, r["n_rad"], r["n_ang"], r["becke_cutoff"]))
            p.name, p.xc = "mol%d" % j, xc
        else:
            p = batch_member(int(n), j, r["n_rad"], r["n_ang"], xc, r["becke_cutoff"])
            if cache:
                _save(p, path)
        out.append(p)
    return out
