"""Seeded synthetic inputs for the implicit M1 radiation step.

This module only draws and lays out input fields (states, opacities, heat
capacities, boundary planes); it holds none of the scheme's arithmetic, so the
CPU oracle and the GPU path can both consume it without sharing method code.

Conventions shared by every generator
-------------------------------------
* Grid sizes are given as ``n = (nx, ny)`` or ``(nx, ny, nz)``; numpy arrays are
  shaped ``(ny, nx)`` / ``(nz, ny, nx)`` (x fastest, the layout the C ABI uses).
* Units are nondimensional: c = a_r = dx = 1, so sigma is the optical depth of
  one cell and the explicit light-crossing step dt_CFL = dx / c = 1.
* A problem is a plain ``dict``:
  ``ndim, n, dx, c, a_r, dt, source, flux_source, closure, ap, lambda_floor,
  bc (6 names: -x,+x,-y,+y,-z,+z), ghost {face: (1+ndim, *plane)},
  ghost_mask {face: plane}, sigma, rho_cv, E, F (ndim, *grid), T``.
* Every random number comes from ``numpy.random.default_rng(seed)`` (PCG64) in
  the draw order written in each docstring.
"""
from __future__ import annotations

import numpy as np

FACE_NAMES = ("-x", "+x", "-y", "+y", "-z", "+z")


def grid_shape(n):
    """numpy shape of a grid with sizes n = (nx, ny[, nz])."""
    return tuple(int(v) for v in reversed(n))


def plane_shape(n, d):
    """numpy shape of a boundary plane normal to direction d (0=x, 1=y, 2=z)."""
    g = list(grid_shape(n))
    del g[len(n) - 1 - d]
    return tuple(g)


def base_problem(n, *, dt, source="none", flux_source="wb", closure="m1",
                 ap=True, lambda_floor=0.0, bc=None, dx=1.0, c=1.0, a_r=1.0):
    ndim = len(n)
    if bc is None:
        bc = ["periodic"] * (2 * ndim)
    bc = list(bc) + ["periodic"] * (6 - len(bc))
    return dict(ndim=ndim, n=tuple(int(v) for v in n), dx=float(dx), c=float(c),
                a_r=float(a_r), dt=float(dt), source=source, flux_source=flux_source,
                closure=closure, ap=bool(ap), lambda_floor=float(lambda_floor),
                bc=bc, ghost={}, ghost_mask={})


def n_unknowns(p):
    return 1 + p["ndim"] + (1 if p["source"] == "coupled_t" else 0)


# --------------------------------------------------------------------------
# Random states for parity tests
# --------------------------------------------------------------------------
def random_problem(n, seed, *, source="none", flux_source="wb", bc=None,
                   dt=3.0, fmax=0.9, sigma_range=(1e-2, 1e2), ap=True,
                   lambda_floor=0.0, closure="m1"):
    """Random but admissible inputs on a grid of sizes n.

    Draw order: E ~ U[0.5, 2]; f ~ U[0, fmax]; direction ~ normal(ndim), normalised;
    log10 sigma ~ U[log10 lo, log10 hi]; T ~ U[0.5, 2]; rho_cv ~ U[0.5, 2];
    then, per Dirichlet face in -x..+z order, ghost E ~ U[0.5, 2], ghost f ~
    U[0, fmax], ghost direction ~ normal; then a second state (the time-n
    state) drawn the same way for E, f, direction and T.
    """
    p = base_problem(n, dt=dt, source=source, flux_source=flux_source, bc=bc,
                     ap=ap, lambda_floor=lambda_floor, closure=closure)
    rng = np.random.default_rng(seed)
    g = grid_shape(n)
    ndim = len(n)

    def draw_state(shape):
        E = rng.uniform(0.5, 2.0, size=shape)
        f = rng.uniform(0.0, fmax, size=shape)
        v = rng.standard_normal(size=(ndim,) + shape)
        v /= np.sqrt((v * v).sum(axis=0))[None]
        F = p["c"] * E[None] * f[None] * v
        return E, F

    E, F = draw_state(g)
    lo, hi = np.log10(sigma_range[0]), np.log10(sigma_range[1])
    p["sigma"] = 10.0 ** rng.uniform(lo, hi, size=g)
    T = rng.uniform(0.5, 2.0, size=g)
    p["rho_cv"] = rng.uniform(0.5, 2.0, size=g)
    for face, name in enumerate(p["bc"][: 2 * ndim]):
        if name == "dirichlet":
            Eg, Fg = draw_state(plane_shape(n, face // 2))
            p["ghost"][face] = np.concatenate([Eg[None], Fg], axis=0)
    En, Fn = draw_state(g)
    Tn = rng.uniform(0.5, 2.0, size=g)
    p["E"], p["F"] = E, F
    p["T"] = T if source == "coupled_t" else None
    p["En"], p["Fn"] = En, Fn
    p["Tn"] = Tn if source == "coupled_t" else None
    return p


def edge_problem(n, seed, *, source="none", flux_source="wb", bc=None, dt=3.0,
                 sigma_range=(1e-2, 1e2)):
    """Random inputs that reach the closure's guard branches.

    Starts from random_problem(n, seed, fmax=0.9, ...) and then, for the
    linearisation state and for the time-n state alike, with one generator
    (seed + 7919) in this draw order: a per-cell class u ~ U[0, 1) and, per cell,
    a reduced-flux magnitude g ~ U[0.9, 3] and an energy e ~ U[0, 0.5].  Classes:
      u < 0.25          : |F| = g c E (super-luminal flux, clamped by the closure)
      0.25 <= u < 0.35  : F = 0 exactly
      0.35 <= u < 0.42  : E = -e (non-positive energy, F kept)
      0.42 <= u < 0.45  : E = 0 exactly
    Then two stripes of reduced flux exactly 1, tangent to the faces between
    them: the cells of columns x = nx//3 and nx//3 + 1 carry F = c E along y (2D),
    or the cells of planes z = nz//3 and nz//3 + 1 carry F = c E along z (3D), so
    the faces between two such cells have both wave speeds zero on both sides.
    """
    p = random_problem(n, seed, source=source, flux_source=flux_source, bc=bc, dt=dt, fmax=0.9,
                       sigma_range=sigma_range)
    rng = np.random.default_rng(seed + 7919)
    ndim = len(n)
    g_shape = grid_shape(n)

    def modify(E, F):
        E = E.copy()
        F = F.copy()
        u = rng.uniform(0.0, 1.0, size=g_shape)
        g = rng.uniform(0.9, 3.0, size=g_shape)
        e = rng.uniform(0.0, 0.5, size=g_shape)
        mag = np.sqrt((F * F).sum(axis=0))
        unit = np.where(mag > 0, F / np.where(mag > 0, mag, 1.0), 0.0)
        sup = u < 0.25
        F[:, sup] = (p["c"] * g * E)[sup] * unit[:, sup]
        F[:, (u >= 0.25) & (u < 0.35)] = 0.0
        neg = (u >= 0.35) & (u < 0.42)
        E[neg] = -e[neg]
        E[(u >= 0.42) & (u < 0.45)] = 0.0
        if ndim == 2:
            i0 = n[0] // 3
            for i in (i0, min(i0 + 1, n[0] - 1)):
                E[:, i] = rng.uniform(0.5, 2.0, size=E.shape[0])
                F[:, :, i] = 0.0
                F[1, :, i] = p["c"] * E[:, i]
        else:
            k0 = n[2] // 3
            for k in (k0, min(k0 + 1, n[2] - 1)):
                E[k] = rng.uniform(0.5, 2.0, size=E.shape[1:])
                F[:, k] = 0.0
                F[2, k] = p["c"] * E[k]
        return E, F

    p["E"], p["F"] = modify(p["E"], p["F"])
    p["En"], p["Fn"] = modify(p["En"], p["Fn"])
    return p


def random_vector(n_total, seed):
    """A seeded standard-normal vector (for operator / preconditioner probes)."""
    return np.random.default_rng(seed).standard_normal(n_total)


# --------------------------------------------------------------------------
# The five workload recipes
# --------------------------------------------------------------------------
def diffusive_gaussian(n=(64, 64), sigma=1e3, width=8.0, amplitude=1.0,
                       floor=1e-6, dt=100.0):
    """2D uniform-opacity diffusive Gaussian (64x64, sigma*dx=1e3, dt=100).

    No random numbers. E = floor + amplitude*exp(-r^2/(2 width^2)) centred on the
    grid centre in cell-corner coordinates (cell centres at i+1/2), so the field
    is exactly mirror symmetric; F = 0; periodic boundaries; radiation only.
    """
    p = base_problem(n, dt=dt)
    nx, ny = n
    x = np.arange(nx) + 0.5 - nx / 2.0
    y = np.arange(ny) + 0.5 - ny / 2.0
    r2 = x[None, :] ** 2 + y[:, None] ** 2
    p["E"] = floor + amplitude * np.exp(-r2 / (2.0 * width ** 2))
    p["F"] = np.zeros((2,) + p["E"].shape)
    p["sigma"] = np.full(p["E"].shape, float(sigma))
    p["rho_cv"] = None
    p["T"] = None
    return p


def beam_shadow(n=(1024, 1024), seed=2011, nclumps=8, sigma_bg=1e-3,
                sigma_clump=1e3, dt=50.0, floor=1e-6, flux_source="centered",
                lambda_floor=0.1):
    """2D beam/shadow: background sigma, random elliptical clumps, left beam.

    Draw order (seed 2011): for each of the nclumps clumps in turn: centre
    x ~ U[0.2, 0.9]*nx, centre y ~ U[0, ny), semi-axis a ~ U[20, 80],
    semi-axis b ~ U[20, 80], angle ~ U[0, pi).  Edges are sharp and overlaps take
    sigma_clump.  The -x face is Dirichlet with E = 1, F = (cE, 0) (reduced flux
    exactly 1, a beam entering the box); the other faces are outflow.
    E0 = floor, F0 = 0, radiation only.

    Scheme settings follow the paper's shadow test (Sect. 5.4): the centred flux
    source (Eq. "wb_naive") and HLL speeds floored at +-0.1 c.  (With the well-
    balanced source, the root of this configuration has E < 0 and an odd-even
    flux mode inside the sharp thick clumps.)
    """
    nx, ny = n
    p = base_problem(n, dt=dt, flux_source=flux_source, lambda_floor=lambda_floor,
                     bc=["dirichlet", "outflow", "outflow", "outflow"])
    rng = np.random.default_rng(seed)
    x = np.arange(nx) + 0.5
    y = np.arange(ny) + 0.5
    X, Y = np.meshgrid(x, y)
    sigma = np.full((ny, nx), float(sigma_bg))
    for _ in range(nclumps):
        cx = rng.uniform(0.2, 0.9) * nx
        cy = rng.uniform(0.0, 1.0) * ny
        a = rng.uniform(20.0, 80.0)
        b = rng.uniform(20.0, 80.0)
        th = rng.uniform(0.0, np.pi)
        dx_, dy_ = X - cx, Y - cy
        u = (dx_ * np.cos(th) + dy_ * np.sin(th)) / a
        v = (-dx_ * np.sin(th) + dy_ * np.cos(th)) / b
        sigma[u * u + v * v <= 1.0] = sigma_clump
    p["sigma"] = sigma
    p["E"] = np.full((ny, nx), float(floor))
    p["F"] = np.zeros((2, ny, nx))
    p["T"] = None
    p["rho_cv"] = None
    ghost = np.zeros((3, ny))
    ghost[0] = 1.0
    ghost[1] = p["c"] * 1.0
    p["ghost"][0] = ghost
    return p


def beam45(n=128, dt=0.5, lambda_floor=0.0, t_background=0.3, t_beam=1.0):
    """2D beam at 45 degrees in vacuum (Sect. 5.3): no randomness.

    The box [-1, 1]^2 on n x n cells (here in cell units, dx = 1), sigma = 0,
    radiation only.  Initial state E = a_r t_background^4 (300 K against a 1000 K
    beam: t_background = 0.3 in units of the beam temperature), F = 0.  The -x
    face is Dirichlet: on the cells with y in [-0.875, -0.75] (rows n/16 .. n/8 - 1,
    8 cells at n = 128) the ghost holds E = a_r t_beam^4 and F = c E (1, 1)/sqrt 2
    (reduced flux 1 along the diagonal); on the rest of that face the ghost holds
    the background state.  The other faces are outflow.  Centred flux source
    (sigma = 0 makes the source choice immaterial).  lambda_floor = 1 gives the
    fixed eigenvalues +-c of the paper's comparison.  dt = 0.5 is the explicit
    CFL limit c dt = dx / 2 of the 2D scheme.
    """
    p = base_problem((n, n), dt=dt, flux_source="centered", lambda_floor=lambda_floor,
                     bc=["dirichlet", "outflow", "outflow", "outflow"])
    e_bg = p["a_r"] * t_background ** 4
    e_beam = p["a_r"] * t_beam ** 4
    rows = np.arange(n)
    on = ((rows >= n // 16) & (rows < n // 8)).astype(float)
    ghost = np.zeros((3, n))
    ghost[0] = e_bg + (e_beam - e_bg) * on
    ghost[1] = ghost[2] = p["c"] * e_beam * on / np.sqrt(2.0)
    p["ghost"][0] = ghost
    p["sigma"] = np.zeros((n, n))
    p["rho_cv"] = None
    p["E"] = np.full((n, n), e_bg)
    p["F"] = np.zeros((2, n, n))
    p["T"] = None
    return p


def marshak_1d(n=400, sigma_dx=25.0, rho_cv=1.0, t0=0.3, t_source=1.0, dt=1e4, ap=True):
    """1D Marshak wave (Sect. 5.1) on an n x 1 grid (y periodic), no randomness.

    Constant sigma (sigma dx = 25 as in the paper) and rho c_v; gas and radiation
    start in equilibrium at t0 (E = a_r t0^4, F = 0); the -x face is Dirichlet
    with E = a_r t_source^4, F = 0 (the source lit at t = 0), the +x face outflow.
    Nondimensional (c = a_r = dx = 1): in the paper's CGS units the radiation
    could not heat the gas within the quoted time, so only the comparison AP
    against plain HLL carries over.  Well-balanced flux source; ap toggles the
    asymptotic correction (ap = False is the standard HLL scheme).
    """
    p = base_problem((n, 1), dt=dt, source="coupled_t", flux_source="wb", ap=ap,
                     bc=["dirichlet", "outflow", "periodic", "periodic"])
    p["sigma"] = np.full((1, n), float(sigma_dx) / p["dx"])
    p["rho_cv"] = np.full((1, n), float(rho_cv))
    p["E"] = np.full((1, n), p["a_r"] * t0 ** 4)
    p["F"] = np.zeros((2, 1, n))
    p["T"] = np.full((1, n), float(t0))
    p["ghost"][0] = np.array([[p["a_r"] * t_source ** 4], [0.0], [0.0]])
    return p


def opacity_jump_1d(n=100, sigma_dx=100.0, t0=0.3, t_source=1.0, dt=1e5, flux_source="wb"):
    """Steady state across a jump of opacity (Sect. 5.2) on an n x 1 grid.

    sigma dx = 100 on the left half (the paper's 10^4 cm^-1 at dx = 0.01 cm) and
    0 on the right half; radiation only (at the steady state the exchange with
    the gas vanishes, so the flux must be constant in x either way); E0 =
    a_r t0^4, F0 = 0; -x face Dirichlet E = a_r t_source^4, F = 0; +x outflow.
    flux_source: "wb" (Eq. "wb_smart") or "centered" (Eq. "wb_naive").
    """
    p = base_problem((n, 1), dt=dt, source="none", flux_source=flux_source,
                     bc=["dirichlet", "outflow", "periodic", "periodic"])
    p["sigma"] = np.where(np.arange(n) < n // 2, float(sigma_dx) / p["dx"], 0.0)[None, :]
    p["rho_cv"] = None
    p["E"] = np.full((1, n), p["a_r"] * t0 ** 4)
    p["F"] = np.zeros((2, 1, n))
    p["T"] = None
    p["ghost"][0] = np.array([[p["a_r"] * t_source ** 4], [0.0], [0.0]])
    return p


def gaussian_random_field(shape, seed, slope=-11.0 / 3.0):
    """Zero-mean, unit-variance periodic Gaussian random field.

    White noise ~ normal(shape) from default_rng(seed), filtered in Fourier space
    by sqrt(P(k)) with P(k) = k**slope for 1 <= |k| <= N/2 (k in integer
    wavenumbers, the k=0 mode and modes beyond the Nyquist radius removed).
    """
    rng = np.random.default_rng(seed)
    w = rng.standard_normal(size=shape)
    wk = np.fft.rfftn(w)
    ks = [np.fft.fftfreq(s) * s for s in shape[:-1]] + [np.fft.rfftfreq(shape[-1]) * shape[-1]]
    grids = np.meshgrid(*ks, indexing="ij")
    k = np.sqrt(sum(g * g for g in grids))
    kmax = min(shape) / 2.0
    amp = np.zeros_like(k)
    sel = (k >= 1.0) & (k <= kmax)
    amp[sel] = k[sel] ** (slope / 2.0)
    g = np.fft.irfftn(wk * amp, s=shape)
    g -= g.mean()
    g /= g.std()
    return g


def coupled_lognormal(n=(256, 256, 256), seeds=(13926, 13927), dt=100.0,
                      sigma0=1.0, sigma_ln=1.0):
    """3D radiation-matter coupling on a lognormal density (gas-temperature row).

    rho = exp(sigma_ln*g1 - sigma_ln^2/2) with g1 the GRF of seed 13926 (mean 1);
    T = 10**(-2 + 3u), u = Phi(g2) with g2 the GRF of seed 13927 (T/1e3 K spans
    1e-2..10, i.e. 10 K..1e4 K); E0 = a_r T^4 (local equilibrium), F0 = 0;
    sigma = sigma0 * rho * T**-3.5; rho_cv = rho (c_v = 1); periodic.
    """
    from scipy.special import ndtr

    p = base_problem(n, dt=dt, source="coupled_t",
                     bc=["periodic"] * 6)
    shape = grid_shape(n)
    g1 = gaussian_random_field(shape, seeds[0])
    g2 = gaussian_random_field(shape, seeds[1])
    rho = np.exp(sigma_ln * g1 - 0.5 * sigma_ln ** 2)
    T = 10.0 ** (-2.0 + 3.0 * ndtr(g2))
    p["T"] = T
    p["E"] = p["a_r"] * T ** 4
    p["F"] = np.zeros((3,) + shape)
    p["sigma"] = sigma0 * rho * T ** -3.5
    p["rho_cv"] = rho
    return p


def diffusive_lognormal(n=(256, 256), seed=0, dt=1000.0, sigma_range=(3.0, 300.0), ngauss=6, floor=1e-6):
    """2D periodic optically thick medium with a smooth opacity field.

    log sigma = log lo + (log hi - log lo) Phi(g), g the k^(-11/3) Gaussian random
    field of `seed` (unit variance), Phi the normal CDF; then, with
    numpy.random.default_rng(seed + 7919), for each of ngauss energy bumps:
    centre x ~ U[0, nx), centre y ~ U[0, ny), width ~ U[4, 16], log10 amplitude
    ~ U[0, 2].  E = floor + bumps, F = 0, radiation only, well-balanced source.
    At dt = 1000 the diffusion length sqrt(c dt / 3 sigma) spans 1-10 cells.
    """
    from scipy.special import ndtr

    nx, ny = n
    p = base_problem(n, dt=dt)
    g = gaussian_random_field(grid_shape(n), seed)
    g = g / max(float(g.std()), 1e-300)
    lo, hi = np.log10(sigma_range[0]), np.log10(sigma_range[1])
    p["sigma"] = 10.0 ** (lo + (hi - lo) * ndtr(g))
    rng = np.random.default_rng(seed + 7919)
    x = np.arange(nx) + 0.5
    y = np.arange(ny) + 0.5

    def pdist(a, b, L):
        d = np.abs(a - b)
        return np.minimum(d, L - d)

    E = np.full((ny, nx), float(floor))
    for _ in range(ngauss):
        cx = rng.uniform(0, nx)
        cy = rng.uniform(0, ny)
        w = rng.uniform(4.0, 16.0)
        amp = 10.0 ** rng.uniform(0.0, 2.0)
        E += amp * np.exp(-(pdist(x[None, :], cx, nx) ** 2 + pdist(y[:, None], cy, ny) ** 2) / (2 * w * w))
    p["E"] = E
    p["F"] = np.zeros((2, ny, nx))
    p["T"] = None
    p["rho_cv"] = None
    return p


def voronoi_opacity(n=(512, 512), seed=0, nsites=64, ngauss=4, dt=100.0, floor=1e-6):
    """2D periodic Voronoi opacity field with Gaussian energy bumps.

    Draw order: site x ~ U[0, nx) and y ~ U[0, ny) for each of nsites sites
    (x array then y array); log10 sigma per site ~ U[-3, 4]; then for each of
    ngauss bumps: centre x ~ U[0, nx), centre y ~ U[0, ny), width ~ U[8, 32],
    log10 amplitude ~ U[0, 2].  Distances are periodic.  F0 = 0, radiation only.
    """
    nx, ny = n
    p = base_problem(n, dt=dt)
    rng = np.random.default_rng(seed)
    sx = rng.uniform(0, nx, size=nsites)
    sy = rng.uniform(0, ny, size=nsites)
    lsig = rng.uniform(-3.0, 4.0, size=nsites)
    x = np.arange(nx) + 0.5
    y = np.arange(ny) + 0.5

    def pdist(a, b, L):
        d = np.abs(a - b)
        return np.minimum(d, L - d)

    best = np.full((ny, nx), np.inf)
    owner = np.zeros((ny, nx), dtype=np.int64)
    for s in range(nsites):
        d2 = pdist(x[None, :], sx[s], nx) ** 2 + pdist(y[:, None], sy[s], ny) ** 2
        closer = d2 < best
        best[closer] = d2[closer]
        owner[closer] = s
    p["sigma"] = 10.0 ** lsig[owner]
    E = np.full((ny, nx), float(floor))
    for _ in range(ngauss):
        cx = rng.uniform(0, nx)
        cy = rng.uniform(0, ny)
        s = rng.uniform(8.0, 32.0)
        amp = 10.0 ** rng.uniform(0.0, 2.0)
        d2 = pdist(x[None, :], cx, nx) ** 2 + pdist(y[:, None], cy, ny) ** 2
        E += amp * np.exp(-d2 / (2 * s * s))
    p["E"] = E
    p["F"] = np.zeros((2, ny, nx))
    p["T"] = None
    p["rho_cv"] = None
    return p


def ionization_front(n=(192, 192, 192), seed=192, dt=100.0, sigma0=1e-2,
                     jump=1e4, patch=4, floor=1e-6, with_velocity=False, mach=0.5, sound_speed=3.3e-5):
    """3D ionisation-front-like absorption run.

    rho: lognormal from the GRF of `seed` (as the coupled workload, sigma_ln=1).
    sigma = sigma0*rho for z < nz/2 and jump*sigma0*rho beyond (planar jump).
    Point source: on the -z face a patch x patch block of cells at the face
    centre is Dirichlet with E = 1, F = (0, 0, cE); the rest of that face and
    all other faces are outflow (ghost_mask 1 on the patch, 0 elsewhere).
    E0 = floor, F0 = 0, absorption source (no gas-temperature row).
    If with_velocity, a solenoidal velocity v = curl A (A: three GRFs of seeds
    seed+1..seed+3) scaled to rms Mach `mach` at the sound speed `sound_speed`
    (in units of c; 3.3e-5 c is 10 km/s, ionised gas) is attached as p['velocity'];
    the implicit radiation step does not use it (hydrodynamics is frozen).
    """
    nx, ny, nz = n
    p = base_problem(n, dt=dt, source="absorption",
                     bc=["outflow", "outflow", "outflow", "outflow", "dirichlet", "outflow"])
    shape = grid_shape(n)
    g = gaussian_random_field(shape, seed)
    rho = np.exp(g - 0.5)
    zc = np.arange(nz)[:, None, None] + 0.5
    sigma = sigma0 * rho * np.where(zc < nz / 2.0, 1.0, jump)
    p["sigma"] = sigma
    p["E"] = np.full(shape, float(floor))
    p["F"] = np.zeros((3,) + shape)
    p["T"] = None
    p["rho_cv"] = None
    ghost = np.zeros((4, ny, nx))
    mask = np.zeros((ny, nx))
    j0, i0 = ny // 2 - patch // 2, nx // 2 - patch // 2
    mask[j0:j0 + patch, i0:i0 + patch] = 1.0
    ghost[0] = mask * 1.0
    ghost[3] = mask * p["c"]
    p["ghost"][4] = ghost
    p["ghost_mask"][4] = mask
    if with_velocity:
        A = [gaussian_random_field(shape, seed + 1 + k) for k in range(3)]
        # curl on the periodic grid by central differences (axes z, y, x)
        def dd(f, ax):
            return 0.5 * (np.roll(f, -1, ax) - np.roll(f, 1, ax))
        vx = dd(A[2], 1) - dd(A[1], 0)
        vy = dd(A[0], 0) - dd(A[2], 2)
        vz = dd(A[1], 2) - dd(A[0], 1)
        rms = np.sqrt((vx ** 2 + vy ** 2 + vz ** 2).mean())
        p["velocity"] = np.stack([vx, vy, vz]) * (mach * sound_speed / rms)
    return p


def window(p, origin, size, bc):
    """A rectangular window of a 2D problem's fields as a problem of its own.

    origin = (i0, j0), size = (nx, ny) in cells; bc: the window's boundary kinds
    (4 names).  sigma, E and F are copied from the window; the scheme settings
    and dt are the parent's.  Used for reduced instances of a large workload
    (the CPU oracle's timing sample); Dirichlet planes of the parent are not
    carried over.
    """
    i0, j0 = origin
    nx, ny = size
    q = base_problem((nx, ny), dt=p["dt"], source=p["source"], flux_source=p["flux_source"],
                     closure=p.get("closure", "m1"), ap=p["ap"], lambda_floor=p["lambda_floor"], bc=list(bc),
                     dx=p["dx"], c=p["c"], a_r=p["a_r"])
    sl = (slice(j0, j0 + ny), slice(i0, i0 + nx))
    q["sigma"] = np.array(p["sigma"][sl], dtype=float)
    q["E"] = np.array(p["E"][sl], dtype=float)
    q["F"] = np.array(p["F"][(slice(None),) + sl], dtype=float)
    q["T"] = None if p.get("T") is None else np.array(p["T"][sl], dtype=float)
    q["rho_cv"] = None if p.get("rho_cv") is None else np.array(p["rho_cv"][sl], dtype=float)
    return q


WORKLOADS = {
    "diffusive_gaussian_64": lambda: diffusive_gaussian(),
    "beam_shadow_1024": lambda: beam_shadow(),
    "coupled_lognormal_256": lambda: coupled_lognormal(),
    "voronoi_512": lambda: voronoi_opacity(),
    "ionization_front_192": lambda: ionization_front(),
}
