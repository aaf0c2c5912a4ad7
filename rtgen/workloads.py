"""Named synthetic workloads (scene + transmitters + launched rays).

* ``microcell``: 200 x 200 m, 242 triangles, Tx (0, 0, 10), level-5
  icosphere (10,242 rays), tmin 1e-4 m, tmax 500 m, one closest-hit segment.
* ``city24k``: 2 x 2 km, 2,000 buildings (about 24k triangles), Tx (0, 0, 25),
  level-9 icosphere (2,621,442 rays), tmin 1e-4 m, tmax 2 km per segment, up to
  6 segments (bounces).
* ``dense200k``: 3 x 3 km, tessellated facades (>= 200k triangles), 4 Tx at
  (+-750, +-750, 25), level 9 per Tx (10,485,768 rays), up to 6 segments.
* ``multiscene``: 8 city scenes of uneven size with 8 Tx each.

The split parameters carry the paper's spatial-distance source point: the
transmitter the BVH is built for (Eq. 2).
"""
from __future__ import annotations

import dataclasses
import functools
import math

import numpy as np

from . import icosphere, scenes


@dataclasses.dataclass
class Workload:
    name: str
    tris: np.ndarray            # float32 [n, 9]
    rays: np.ndarray            # float32 [m, 8]
    tx: tuple                   # source point used for the distance term
    max_bounces: int
    tmin: float
    tmax: float
    level: int

    @property
    def n_tris(self) -> int:
        return int(self.tris.shape[0])

    @property
    def n_rays(self) -> int:
        return int(self.rays.shape[0])


@functools.lru_cache(maxsize=2)
def _city24k_tris(seed: int) -> np.ndarray:
    return scenes.city(seed=seed)


@functools.lru_cache(maxsize=1)
def _dense_tris(seed: int) -> np.ndarray:
    return scenes.dense_city(seed=seed)


def microcell(seed: int = 0) -> Workload:
    tx = (0.0, 0.0, 10.0)
    tris = scenes.microcell(seed=seed, tx=tx)
    rays = icosphere.make_rays(tx, icosphere.directions(5), 1e-4, 500.0)
    return Workload("microcell-242tri-L5", tris, rays, tx, 1, 1e-4, 500.0, 5)


def city24k(seed: int = 0, level: int = 9, max_bounces: int = 6) -> Workload:
    tx = (0.0, 0.0, 25.0)
    tris = _city24k_tris(seed)
    rays = icosphere.make_rays(tx, icosphere.directions(level), 1e-4, 2000.0)
    return Workload(f"city-{tris.shape[0]}tri-L{level}-b{max_bounces}", tris, rays,
                    tx, max_bounces, 1e-4, 2000.0, level)


DENSE_TX = ((-750.0, -750.0, 25.0), (750.0, -750.0, 25.0),
            (-750.0, 750.0, 25.0), (750.0, 750.0, 25.0))


def dense200k(seed: int = 0, level: int = 9, max_bounces: int = 6) -> Workload:
    """Rays of the 4 transmitters concatenated; the distance term uses the
    centre of the four (the BVH serves all of them at once)."""
    tris = _dense_tris(seed)
    d = icosphere.directions(level)
    rays = np.concatenate([icosphere.make_rays(t, d, 1e-4, 2000.0) for t in DENSE_TX])
    centre = tuple(float(np.mean([t[i] for t in DENSE_TX])) for i in range(3))
    return Workload(f"dense-{tris.shape[0]}tri-4xL{level}-b{max_bounces}", tris, rays,
                    centre, max_bounces, 1e-4, 2000.0, level)


MULTI_TARGETS = (1_000, 4_000, 12_000, 24_000, 50_000, 90_000, 140_000, 200_000)


def multiscene_scene(i: int) -> tuple[np.ndarray, float]:
    """Scene i of the uneven multi-scene set: ``target / 12`` buildings on a
    square of side 2 km * sqrt(target / 24k), seed i; returns (tris, half)."""
    target = MULTI_TARGETS[i]
    nb = max(1, target // 12)
    half = 1000.0 * math.sqrt(target / 24_000)
    return scenes.city(seed=i, n_buildings=nb, half=half, tx=None), half


def multiscene_queries(seed: int = 0, per_scene: int = 8, levels=(6, 9), bounces=(1, 6)):
    """Transmitters spread over the 8 scenes: per query (scene, tx, level,
    max_bounces); Tx uniform outside buildings at 25 m."""
    rng = np.random.default_rng(1000 + seed)
    out = []
    for s in range(len(MULTI_TARGETS)):
        tris, half = multiscene_scene(s)
        for _ in range(per_scene):
            tx = scenes.free_point(rng, half, tris, 25.0)
            lv = int(rng.integers(levels[0], levels[1] + 1))
            nb = int(rng.integers(bounces[0], bounces[1] + 1))
            out.append((s, tx, lv, nb))
    return out


# Trees of the multi-scene set are built once per scene with the ray source
# point at the scene centre, 25 m up; queries bring their own transmitters.
MULTI_SRC = (0.0, 0.0, 25.0)


def multiscene_rays(tx, level: int) -> np.ndarray:
    """Rays of one multi-scene query: the level's icosphere from tx,
    tmin 1e-4 m, tmax 2 km."""
    return icosphere.make_rays(tx, icosphere.directions(level), 1e-4, 2000.0)


def reception_chains(seed: int = 0, groups: int = 600, per_group: int = 8, max_b: int = 4,
                     n_rx: int = 256, n_ids: int = 3):
    """Synthetic stored chains and field points for the receiving-sphere test.

    Rays come in groups of ``per_group`` nearly identical chains (the base
    chain's float64 origins and directions moved by up to 1e-3 relative, the
    same facet ids, hit parameters moved by up to 1e-3), so that several rays
    of a group pass near the same field point, as neighbouring launched rays
    do.  Per segment of a base chain, in draw order: origin ~ U(-50, 50)^3,
    direction ~ N(0, 1)^3 scaled to a length ~ U(0.5, 2), tmin ~ U(0, 0.01),
    tmax ~ U(50, 200), hit with probability 0.7 at t ~ U(tmin + 1, tmax) on
    facet ~ U{0 .. n_ids - 1}.  A chain ends at its first miss; rows of
    segments never traced are NaN with id -1 and t = +inf.

    Field points: each picks a random existing segment of a random base
    chain, a parameter s ~ U(t0 - 5 %, t1 + 5 %) of its range and an offset
    perpendicular to it of length ~ U(0, 4) m.

    Returns (seg float32 [max_b, m, 8], hit_id int32 [max_b, m],
    hit_t float32 [max_b, m], receivers float64 [n_rx, 3]), m = groups *
    per_group.
    """
    rng = np.random.default_rng(seed)
    m = groups * per_group
    seg = np.full((max_b, m, 8), np.nan, np.float32)
    hid = np.full((max_b, m), -1, np.int32)
    ht = np.full((max_b, m), np.inf, np.float32)
    base = []
    for g in range(groups):
        chain = []
        for b in range(max_b):
            o = rng.uniform(-50, 50, 3)
            d = rng.normal(size=3)
            d *= rng.uniform(0.5, 2.0) / np.linalg.norm(d)
            t0, t1 = rng.uniform(0, 0.01), rng.uniform(50, 200)
            hit = rng.uniform() < 0.7
            t = rng.uniform(t0 + 1, t1)
            fid = int(rng.integers(0, n_ids))
            chain.append((o, d, t0, t1, hit, t, fid))
            if not hit:
                break
        base.append(chain)
        for k in range(per_group):
            i = g * per_group + k
            for b, (o, d, t0, t1, hit, t, fid) in enumerate(chain):
                jo = o * (1 + rng.uniform(-1e-3, 1e-3, 3)) if k else o
                jd = d * (1 + rng.uniform(-1e-3, 1e-3, 3)) if k else d
                seg[b, i] = [*jo, t0, *jd, t1]
                if hit:
                    hid[b, i] = fid
                    ht[b, i] = t * (1 + rng.uniform(-1e-3, 1e-3)) if k else t
    rx = np.empty((n_rx, 3))
    for r in range(n_rx):
        chain = base[int(rng.integers(0, groups))]
        o, d, t0, t1, hit, t, _ = chain[int(rng.integers(0, len(chain)))]
        end = t if hit else t1
        s = rng.uniform(t0 - 0.05 * (end - t0), end + 0.05 * (end - t0))
        p = rng.normal(size=3)
        p -= d * (p @ d) / (d @ d)
        p *= rng.uniform(0, 4.0) / np.linalg.norm(p)
        rx[r] = o + s * d + p
    return seg, hid, ht, rx


def field_points(tris: np.ndarray, half: float, n: int, seed: int) -> np.ndarray:
    """n receiver positions (float64 [n, 3]) outside the buildings: (x, y)
    uniform in the square of half-side 0.95 * half that no roof covers,
    height ~ U(1.5, 30) m drawn before each position."""
    rng = np.random.default_rng(seed)
    pts = [scenes.free_point(rng, half, tris, float(rng.uniform(1.5, 30.0))) for _ in range(n)]
    return np.array(pts, np.float64).reshape(-1, 3)


def normal_incidence_reflection(eps_r: float) -> float:
    """Power reflection coefficient |(1 - sqrt(eps)) / (1 + sqrt(eps))|^2 of a
    lossless dielectric half-space at normal incidence."""
    r = (1.0 - math.sqrt(eps_r)) / (1.0 + math.sqrt(eps_r))
    return r * r


# Power reflection coefficient per material index (scenes.MATERIALS order):
# the paper names the materials but gives no values, so these are illustrative
# inputs -- normal-incidence values for relative permittivities 5.3 (concrete),
# 2.0 (wood) and 6.3 (glass), and 1 for metal (a perfect conductor).
REFLECTION = np.array([normal_incidence_reflection(5.3), normal_incidence_reflection(2.0), 1.0,
                       normal_incidence_reflection(6.3)])
FREQUENCY_HZ = 2.4e9      # the paper's simulation frequency (Sec. IV-A)


def free_space_k0(frequency_hz: float = FREQUENCY_HZ) -> float:
    """(lambda / (4 pi))^2: power ratio between isotropic antennas 1 m apart."""
    lam = 299_792_458.0 / frequency_hz
    return (lam / (4.0 * math.pi)) ** 2


def city_materials(n_tris: int, seed: int = 0) -> np.ndarray:
    """Material index per facet of a city scene: the two ground facets
    concrete, every other facet concrete / glass / metal with probabilities
    0.8 / 0.15 / 0.05 (one draw per facet)."""
    rng = np.random.default_rng(seed)
    u = rng.uniform(size=n_tris)
    m = np.where(u < 0.8, scenes.CONCRETE, np.where(u < 0.95, scenes.GLASS, scenes.METAL))
    m[:2] = scenes.CONCRETE
    return m.astype(np.int32)


@dataclasses.dataclass
class PaperScene:
    """A stand-in for one of the paper's two simulation scenes, with the
    paper's Tx, Rx, leaf threshold, Eq. (2) weight alpha and reflection
    order (Sec. IV-A)."""
    name: str
    tris: np.ndarray
    tx: tuple
    rx: tuple
    max_leaf: int
    alpha: float
    max_order: int       # highest reflection order received
    tmax: float
    material: np.ndarray = None   # int32 [n] material index per facet (scenes.MATERIALS)

    @property
    def max_bounces(self) -> int:
        """Segments per chain: a path with k reflections is received on segment k."""
        return self.max_order + 1

    def rays(self, level: int) -> np.ndarray:
        return icosphere.make_rays(self.tx, icosphere.directions(level), 1e-4, self.tmax)


def paper_indoor(seed: int = 0) -> PaperScene:
    """Study room 8 x 6 x 3.5 m, 2,778 facets; Tx (1.46, 2.42, 2.1), Rx (1.2,
    1.2, 1.5); 250 facets per leaf, alpha 0.7; reflection orders 1 and 2;
    tmax 20 m per segment."""
    tris, mat = scenes.study_room(seed, materials=True)
    return PaperScene("indoor-2778", tris, (1.46, 2.42, 2.1), (1.2, 1.2, 1.5), 250, 0.7, 2, 20.0,
                      mat)


def paper_outdoor(seed: int = 0) -> PaperScene:
    """Campus 1 x 1 km, 7,608 facets; Tx (450, 450, 10), Rx (450, 550, 25);
    820 facets per leaf, alpha 0.4; reflection order 3; tmax 2 km per
    segment."""
    tris, mat = scenes.campus(seed, materials=True)
    return PaperScene("outdoor-7608", tris, (450.0, 450.0, 10.0), (450.0, 550.0, 25.0), 820, 0.4,
                      3, 2000.0, mat)
