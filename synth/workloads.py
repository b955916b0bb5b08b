"""The named workloads: grid, material constants, load history and seeds.

Material constants: cubic FCC elasticity C11/C12/C44 = 168.4/121.4/75.4 GPa,
12 {111}<110> slip systems, power-law flow (reference rate 1e-3/s, exponent 20),
initial strength 50 MPa, linear hardening 200 MPa; phase-field length 2 voxels
and fracture toughness drawn uniformly in [0.5, 1.5] J/m^2 per run.  Constants
the workloads leave open are taken from the paper's Table 1 and its numerical
setup (Burgers vector 3.5e-10 m, SSD coefficient 1.5e14 m^-2, voxel 0.78 um,
strain rate 1e-3/s, regularisation length of the plastic distortion 2 voxels).

Workloads with ``material = 1`` use the paper's thermally activated flow rule with
Taylor hardening and its Table 1 constants (CMSX-4 at room temperature: C11/C12/C44
= 250/161/129 GPa, initial CRSS 350 MPa, b = 3.5e-10 m, v_D = 1e11 1/s,
k = 1.4e-23 J/K, dF = 4.9e-20 J, rho_m = 5e12 1/m^2, lambda = 1.5e14 1/m^2, T = 295 K).
The paper gives neither the activation volume nor the shear modulus of the Taylor
term: dV = 20 b^3 and mu = C44 here.
"""
import dataclasses
import numpy as np

from .microstructure import (periodic_voronoi, periodic_laguerre, shoemake_quaternions,
                             lognormal_laguerre_weights, notch_mask)
from .loading import triangular_waveform

VOXEL = 0.78e-6


@dataclasses.dataclass
class Workload:
    name: str
    n: tuple
    n_grains: int
    seed: int
    amplitude: float
    ratio: int
    cycles: int
    incs_per_cycle: int
    h: float = VOXEL
    laguerre_sigma: float = 0.0       # > 0: log-normal Laguerre cells
    hard_fraction: float = 0.0        # fraction of grains with doubled strength
    notch: bool = False
    # material
    C11: float = 168.4e9
    C12: float = 121.4e9
    C44: float = 75.4e9
    gdot0: float = 1e-3
    n_exp: float = 20.0
    tau_c0: float = 50e6
    h_lin: float = 200e6
    lambda_ssd: float = 1.5e14
    rho0: float = 1e12
    burgers: float = 3.5e-10
    xi_store: float = 0.05
    # phase field
    ell_vox: float = 2.0
    Gc: float = None                  # drawn from the seed when None
    G_crit: float = 4.0
    k_res: float = 1e-5
    ell_fp_vox: float = 2.0
    rate: float = 1e-3
    # thermally activated flow + Taylor hardening (material = 1)
    material: int = 0
    rho_m: float = 5e12
    v_D: float = 1e11
    dF: float = 4.9e-20
    k_B: float = 1.4e-23
    T: float = 295.0
    dV_b3: float = 20.0               # activation volume in units of b^3
    mu: float = None                  # Taylor shear modulus; C44 when None
    # solver (paper's production tolerances by default)
    tol_stag: float = 5e-3
    tol_newton: float = 5e-3
    tol_lin: float = 1e-5
    max_stag: int = 50
    max_newton: int = 100
    max_krylov: int = 500
    gmres_restart: int = 30

    def parity(self):
        """Copy with the tight tolerances under which the discrete solution is unique
        to well below the parity bar."""
        return dataclasses.replace(self, tol_stag=1e-11, tol_newton=1e-11, tol_lin=1e-12,
                                   max_stag=200, max_newton=100, max_krylov=4000)

    @property
    def nvox(self):
        return int(np.prod(self.n))

    @property
    def ell(self):
        return self.ell_vox * self.h

    @property
    def ell_fp(self):
        return self.ell_fp_vox * self.h

    def gc_value(self):
        if self.Gc is not None:
            return float(self.Gc)
        return float(np.random.default_rng(self.seed).uniform(0.5, 1.5))

    def load(self):
        return triangular_waveform(self.amplitude, self.ratio, self.cycles,
                                   self.incs_per_cycle, self.rate)

    def desc(self):
        """Flat dict of every scalar the solver needs (sizes, constants, tolerances)."""
        return dict(n=tuple(self.n), h=self.h, C11=self.C11, C12=self.C12, C44=self.C44,
                    gdot0=self.gdot0, n_exp=self.n_exp, tau_c0=self.tau_c0, h_lin=self.h_lin,
                    lambda_ssd=self.lambda_ssd, rho0=self.rho0, burgers=self.burgers,
                    xi_store=self.xi_store, ell=self.ell, Gc=self.gc_value(),
                    G_crit=self.G_crit, k_res=self.k_res, ell_fp=self.ell_fp,
                    tol_stag=self.tol_stag, tol_newton=self.tol_newton, tol_lin=self.tol_lin,
                    max_stag=self.max_stag, max_newton=self.max_newton,
                    max_krylov=self.max_krylov, gmres_restart=self.gmres_restart,
                    material=int(self.material), rho_m=self.rho_m, v_D=self.v_D, dF=self.dF,
                    k_B=self.k_B, T=self.T, dV=self.dV_b3 * self.burgers ** 3,
                    mu=self.C44 if self.mu is None else self.mu)


def make_inputs(w):
    """Seeded microstructure of a workload.

    Returns dict(grain=int32[N] (x fastest), quat=float64[G,4] (w,x,y,z, crystal->sample),
    tau_c0=float64[G], phi0=float64[N] or None, deps=float64[K], dt=float64[K]).
    Draw order from ``default_rng(seed)``: toughness, seeds, (Laguerre volumes),
    orientations, (hard grains).
    """
    rng = np.random.default_rng(w.seed)
    rng.uniform(0.5, 1.5)                          # the toughness draw (see gc_value)
    g = int(w.n_grains)
    if g == 1:
        grain = np.zeros(w.nvox, dtype=np.int32)
    else:
        seeds = rng.random((g, 3)) * np.array(w.n, dtype=np.float64)
        if w.laguerre_sigma > 0:
            wts = lognormal_laguerre_weights(w.n, g, w.laguerre_sigma, rng)
            grain = periodic_laguerre(w.n, seeds, wts)
        else:
            grain = periodic_voronoi(w.n, seeds)
    quat = shoemake_quaternions(g, rng)
    tau = np.full(g, w.tau_c0)
    if w.hard_fraction > 0:
        nh = int(round(w.hard_fraction * g))
        hard = rng.choice(g, size=nh, replace=False)
        tau[hard] *= 2.0
    phi0 = notch_mask(w.n) if w.notch else None
    deps, dt = w.load()
    return dict(grain=grain, quat=quat, tau_c0=tau, phi0=phi0, deps=deps, dt=dt)


def single_crystal(n=16, seed=0, notch=True, **kw):
    return Workload(name=f"single-crystal-{n}", n=(n, n, n), n_grains=1, seed=seed,
                    amplitude=0.005, ratio=-1, cycles=2, incs_per_cycle=20, notch=notch, **kw)


def cmsx4(**kw):
    """Table 1 constants (thermally activated flow, Taylor hardening) and the paper's
    load: strain ratio 0, amplitude 2 %, strain rate 1e-3/s.  The nearly rate-independent
    slip makes the yielded tangent stiff in some directions and soft in others, so the
    Krylov solves take more iterations: their cap is raised to 3000."""
    base = dict(material=1, C11=250e9, C12=161e9, C44=129e9, tau_c0=350e6, h_lin=0.0,
                amplitude=0.02, ratio=0, max_krylov=3000)
    base.update(kw)
    return base


def small_polycrystal(n=16, n_grains=8, seed=11, **kw):
    base = dict(amplitude=0.006, ratio=0, cycles=3, incs_per_cycle=20)
    base.update(kw)
    nn = n if isinstance(n, tuple) else (n, n, n)
    return Workload(name=f"voronoi-{'x'.join(map(str, nn))}-{n_grains}", n=nn,
                    n_grains=n_grains, seed=seed, **base)


WORKLOADS = {
    # plain FP64, notched single crystal; the oracle finishes in seconds
    # (G_crit lowered from 4 by a power of 2 so that damage starts within the run)
    "notched-crystal-16": Workload(name="notched-crystal-16", n=(16, 16, 16), n_grains=1,
                                   seed=0, amplitude=0.005, ratio=-1, cycles=2,
                                   incs_per_cycle=20, notch=True, G_crit=0.25),
    # plain FP64 polycrystal; damage initiates from the stored energy (G_crit lowered from
    # 4 by powers of 2, to 4 / 2^7 J/m^2, so that it starts within the first cycle)
    "voronoi-64-g64": Workload(name="voronoi-64-g64", n=(64, 64, 64), n_grains=64, seed=1,
                               amplitude=0.006, ratio=0, cycles=3, incs_per_cycle=20,
                               G_crit=4.0 / 2 ** 7),
    # headline: 128^3, 512 log-normal Laguerre grains, fully reversed
    "laguerre-128-g512": Workload(name="laguerre-128-g512", n=(128, 128, 128), n_grains=512,
                                  seed=2, amplitude=0.005, ratio=-1, cycles=2,
                                  incs_per_cycle=20, laguerre_sigma=0.4),
    # at scale: 256^3, 4096 grains, 5% hard grains
    "voronoi-256-g4096-hard": Workload(name="voronoi-256-g4096-hard", n=(256, 256, 256),
                                       n_grains=4096, seed=3, amplitude=0.007, ratio=0,
                                       cycles=2, incs_per_cycle=16, hard_fraction=0.05),
    # a plate one voxel thick (the paper's plate grids, Secs. 4.1-4.3), 64 Voronoi grains,
    # for pointwise plane stress under uniaxial load
    "plate-256-g64": Workload(name="plate-256-g64", n=(256, 256, 1), n_grains=64, seed=7,
                              amplitude=0.006, ratio=0, cycles=3, incs_per_cycle=20),
    # thermally activated flow with Taylor hardening (Table 1): 16^3 Voronoi, 4 grains
    # (the oracle takes about a minute for the first six increments at tight tolerances)
    "cmsx4-voronoi-16-g4": Workload(name="cmsx4-voronoi-16-g4", n=(16, 16, 16), n_grains=4,
                                    seed=3, cycles=1, incs_per_cycle=20, **cmsx4()),
    # thermally activated flow with Taylor hardening (Table 1), 128^3, 512 Laguerre grains
    "cmsx4-laguerre-128-g512": Workload(name="cmsx4-laguerre-128-g512", n=(128, 128, 128),
                                        n_grains=512, seed=5, cycles=1, incs_per_cycle=20,
                                        laguerre_sigma=0.4, **cmsx4()),
}


def workload(name):
    return dataclasses.replace(WORKLOADS[name])
