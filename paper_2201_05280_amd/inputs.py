"""Seeded synthetic input fields (rho, u, theta_T, theta_R) on the bcc grid.

Shared by the tests, the benchmark and the smoke check, for both the HIP path
and the CPU oracle.  Holds no arithmetic of the method itself: only site
positions, analytic initial fields and seeded noise.

Site order of every field: [sub][z][y][x]; sub 0 = corner sites at integer
cell positions (x, y, z), sub 1 = body-centre sites at (x, y, z) + 1/2.
"""
import numpy as np

THETA0 = 0.2948964908710633  # lattice reference temperature (Table of weights)


def positions(nx, ny, nz):
    """(3, 2*nx*ny*nz) site coordinates in units of the cell spacing."""
    sub, z, y, x = np.meshgrid(np.arange(2), np.arange(nz), np.arange(ny), np.arange(nx),
                               indexing="ij")
    off = 0.5 * sub
    return np.stack([(x + off).ravel(), (y + off).ravel(), (z + off).ravel()]).astype(np.float64)


def uniform(nx, ny, nz, rho=1.0, u=(0.0, 0.0, 0.0), theta=THETA0, thetaR=None):
    ns = 2 * nx * ny * nz
    thetaR = theta if thetaR is None else thetaR
    return dict(rho=np.full(ns, float(rho)),
                u=np.tile(np.asarray(u, dtype=np.float64)[:, None], (1, ns)),
                thT=np.full(ns, float(theta)), thR=np.full(ns, float(thetaR)))


def shear_wave(nx, ny, nz, amp=0.01, axis_u=0, axis_k=1, theta=THETA0):
    """u_{axis_u} = amp sin(2 pi x_{axis_k} / n_{axis_k}) at each site's own coordinate."""
    pos = positions(nx, ny, nz)
    n = (nx, ny, nz)[axis_k]
    f = uniform(nx, ny, nz, theta=theta)
    f["u"][axis_u] = amp * np.sin(2 * np.pi * pos[axis_k] / n)
    return f


def density_wave(nx, ny, nz, eps=1e-3, axis=0, theta=THETA0):
    """Isothermal p = p0 (1 + eps cos k x): carried by rho at theta0."""
    pos = positions(nx, ny, nz)
    n = (nx, ny, nz)[axis]
    f = uniform(nx, ny, nz, theta=theta)
    f["rho"] = 1.0 + eps * np.cos(2 * np.pi * pos[axis] / n)
    return f


def temperature_wave(nx, ny, nz, eps=1e-3, axis=0, theta=THETA0):
    """theta = theta0 (1 + eps cos k x) at uniform pressure (rho theta = theta0)."""
    pos = positions(nx, ny, nz)
    n = (nx, ny, nz)[axis]
    f = uniform(nx, ny, nz, theta=theta)
    th = theta * (1.0 + eps * np.cos(2 * np.pi * pos[axis] / n))
    f["thT"] = th.copy()
    f["thR"] = th.copy()
    f["rho"] = theta / th
    return f


def taylor_green(n, U, theta=THETA0, rho0=1.0):
    """3D Taylor-Green vortex on an n^3 periodic box (k = 2 pi / n).

    u =  U sin kx cos ky cos kz,  v = -U cos kx sin ky cos kz,  w = 0,
    p = p0 + rho0 U^2/16 (cos 2kx + cos 2ky)(cos 2kz + 2), carried by rho at theta0.
    """
    pos = positions(n, n, n)
    k = 2 * np.pi / n
    x, y, z = pos * k
    f = uniform(n, n, n, theta=theta)
    f["u"][0] = U * np.sin(x) * np.cos(y) * np.cos(z)
    f["u"][1] = -U * np.cos(x) * np.sin(y) * np.cos(z)
    p = rho0 * theta + rho0 * U * U / 16.0 * (np.cos(2 * x) + np.cos(2 * y)) * (np.cos(2 * z) + 2.0)
    f["rho"] = p / theta
    return f


def random_smooth(nx, ny, nz, seed, amp_rho=0.02, amp_u=0.03, amp_th=0.03, modes=3, theta=THETA0):
    """Seeded sum of a few random Fourier modes in every field, theta_T != theta_R."""
    rng = np.random.default_rng(seed)
    pos = positions(nx, ny, nz)
    n = np.array([nx, ny, nz], dtype=np.float64)[:, None]

    def field(amp):
        out = np.zeros(pos.shape[1])
        for _ in range(modes):
            kk = rng.integers(0, 3, size=3) * (n[:, 0] > 1)
            ph = rng.uniform(0, 2 * np.pi)
            out += amp * rng.uniform(-1, 1) * np.cos((2 * np.pi * kk[:, None] * pos / n).sum(0) + ph)
        return out

    f = uniform(nx, ny, nz, theta=theta)
    f["rho"] = 1.0 + field(amp_rho)
    for a in range(3):
        f["u"][a] = field(amp_u)
    f["thT"] = theta * (1.0 + field(amp_th))
    f["thR"] = theta * (1.0 + field(amp_th))
    return f


MLP_SHAPES = [(128, 6), (128,), (128, 128), (128,), (128, 128), (128,), (128, 128), (128,), (4, 128), (4,)]


def mlp_init(seed):
    """Initial weights of the 6-128-128-128-128-4 coordinate MLP, flat in the
    order W1, b1, ..., W5, b5 (row-major [out][in]): He uniform
    U(-sqrt(6/fan_in), sqrt(6/fan_in)) for weights, zero biases; float32."""
    rng = np.random.default_rng(seed)
    parts = []
    for s in MLP_SHAPES:
        if len(s) == 2:
            lim = np.sqrt(6.0 / s[1])
            parts.append(rng.uniform(-lim, lim, s).ravel())
        else:
            parts.append(np.zeros(s[0]))
    return np.concatenate(parts).astype(np.float32)


def rankine_hugoniot(Ma, gamma, theta1=THETA0, rho1=1.0):
    """Upstream and downstream states (rho, u_x, theta) of a normal shock of an
    ideal gas of heat-capacity ratio gamma, upstream Mach number Ma (flow along
    +x, upstream at low x)."""
    r = (gamma + 1) * Ma ** 2 / ((gamma - 1) * Ma ** 2 + 2)
    p = 1 + 2 * gamma / (gamma + 1) * (Ma ** 2 - 1)
    u1 = Ma * np.sqrt(gamma * theta1)
    return (rho1, u1, theta1), (rho1 * r, u1 / r, theta1 * p / r)


def shock_tube(L, Ma, gamma, theta1=THETA0, width=4.0, x0=None):
    """1D line of L cells holding a tanh blend of the two Rankine-Hugoniot
    states of `rankine_hugoniot`, centred at x0 (default L/2) with the given
    width in cells; theta_R = theta_T."""
    (r1, u1, t1), (r2, u2, t2) = rankine_hugoniot(Ma, gamma, theta1)
    x = positions(L, 1, 1)[0]
    x0 = L / 2 if x0 is None else x0
    sm = 0.5 * (1 + np.tanh((x - x0) / width))
    f = uniform(L, 1, 1)
    f["rho"] = r1 + (r2 - r1) * sm
    f["u"][0] = u1 + (u2 - u1) * sm
    f["thT"] = t1 + (t2 - t1) * sm
    f["thR"] = f["thT"].copy()
    return f
