"""Seeded synthetic inputs (initial fields, solid geometry, particle clouds).

This module holds no arithmetic of the method itself: it only produces the
inputs that both the GPU path and the CPU oracle consume, and the block/node
addressing needed to sample a field at the nodes of a block list.

Addressing conventions (shared by specification, not by code):
  * a block key is the Morton code of its block coordinates (bx, by, bz), x in
    the lowest bit of each 3-bit group;
  * inside a block, node (x, y, z) has index x + 8y + 64z;
  * node n of level l sits at fine-unit position 2^l * n (node-centred levels);
  * moment order (rho - 1, ux, uy, uz, Sxx, Syy, Szz, Sxy, Sxz, Syz).
"""
import numpy as np

PERIODIC, INFLOW, OUTFLOW, WALL, OUTFLOW_CONV = 0, 1, 2, 3, 4


def morton_encode(bx, by, bz):
    bx, by, bz = (np.asarray(v, dtype=np.int64) for v in (bx, by, bz))
    k = np.zeros(np.broadcast(bx, by, bz).shape, dtype=np.int64)
    for bit in range(21):
        k |= ((bx >> bit) & 1) << (3 * bit)
        k |= ((by >> bit) & 1) << (3 * bit + 1)
        k |= ((bz >> bit) & 1) << (3 * bit + 2)
    return k


def morton_decode(keys):
    keys = np.asarray(keys, dtype=np.int64)
    b = [np.zeros_like(keys) for _ in range(3)]
    for bit in range(21):
        for a in range(3):
            b[a] |= ((keys >> (3 * bit + a)) & 1) << bit
    return b[0], b[1], b[2]


_LOCAL = np.stack(np.meshgrid(np.arange(8), np.arange(8), np.arange(8), indexing="ij"), -1)
# node index n = x + 8y + 64z  ->  local (x, y, z)
_LOCAL_XYZ = np.stack([np.arange(512) % 8, (np.arange(512) // 8) % 8, np.arange(512) // 64], -1)


def node_positions(level, keys):
    """Fine-unit positions of every node of the given blocks: int64 [nb, 512, 3]."""
    bx, by, bz = morton_decode(keys)
    base = np.stack([bx, by, bz], -1)[:, None, :] * 8
    return (base + _LOCAL_XYZ[None]) << level


def moments_from_fields(rho_m1, u, S=None):
    """Pack (rho-1, u, S) node arrays into [nb, 10, 512]; S defaults to u u."""
    nb = rho_m1.shape[0]
    out = np.empty((nb, 10, 512), dtype=np.float64)
    out[:, 0] = rho_m1
    for a in range(3):
        out[:, 1 + a] = u[a]
    if S is None:
        S = [u[0] * u[0], u[1] * u[1], u[2] * u[2], u[0] * u[1], u[0] * u[2], u[1] * u[2]]
    for k in range(6):
        out[:, 4 + k] = S[k]
    return out


def uniform_field(level, keys, rho=1.0, u=(0.0, 0.0, 0.0)):
    nb = len(keys)
    r = np.full((nb, 512), rho - 1.0)
    uu = [np.full((nb, 512), float(v)) for v in u]
    return moments_from_fields(r, uu)


def tgv3d_field(level, keys, n, amp=0.05, wavelength=None, pressure=False):
    """3D Taylor-Green vortex: u = U sin kx cos ky cos kz, v = -U cos kx sin ky cos kz,
    w = 0; S = u u; rho = 1, or with pressure=True rho = 1 + 3p with the vortex's
    pressure p = U^2/16 (cos 2kx + cos 2ky)(cos 2kz + 2). k = 2 pi / wavelength (fine
    units, default the x extent)."""
    lam = float(n[0] if wavelength is None else wavelength)
    k = 2.0 * np.pi / lam
    p = node_positions(level, keys).astype(np.float64)
    x, y, z = p[..., 0], p[..., 1], p[..., 2]
    ux = amp * np.sin(k * x) * np.cos(k * y) * np.cos(k * z)
    uy = -amp * np.cos(k * x) * np.sin(k * y) * np.cos(k * z)
    uz = np.zeros_like(ux)
    r = np.zeros_like(ux)
    if pressure:
        r = 3.0 * amp * amp / 16.0 * (np.cos(2 * k * x) + np.cos(2 * k * y)) * (np.cos(2 * k * z) + 2.0)
    return moments_from_fields(r, [ux, uy, uz])


def sample_dense(level, keys, dense):
    """Sample dense fine-unit fields [c, Z, Y, X] at the nodes of the blocks: [nb, c, 512]."""
    p = node_positions(level, keys)
    return dense[:, p[..., 2], p[..., 1], p[..., 0]].transpose(1, 0, 2)


def sphere_solid(n, center, radius):
    """uint8 [Z, Y, X]: 1 where (x-cx)^2 + (y-cy)^2 + (z-cz)^2 <= r^2 (fine units)."""
    z, y, x = np.meshgrid(np.arange(n[2]), np.arange(n[1]), np.arange(n[0]), indexing="ij")
    d2 = (x - center[0]) ** 2 + (y - center[1]) ** 2 + (z - center[2]) ** 2
    return (d2 <= radius * radius).astype(np.uint8)


def slab_particles(count, seed, lo, hi):
    """Uniform random particles (float32 [count, 3]) in the box [lo, hi)."""
    rng = np.random.default_rng(seed)
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    p = lo + (hi - lo) * rng.random((count, 3))
    p = p.astype(np.float32)
    # float32 rounding can land exactly on hi; keep the cloud inside [lo, hi)
    p = np.minimum(p, np.nextafter(hi.astype(np.float32), np.float32(-np.inf)))
    return np.ascontiguousarray(p)


def smooth_random_velocity(n, seed, kmax=6.0, rms=0.03):
    """Divergence-free random velocity [3, Z, Y, X] on a periodic n^3 box: Gaussian noise
    per component, low-passed to integer wavevectors |k| <= kmax, Leray-projected and
    scaled to the given rms over all components."""
    rng = np.random.default_rng(seed)
    shape = (n[2], n[1], n[0])
    noise = rng.standard_normal((3,) + shape)
    F = np.fft.fftn(noise, axes=(1, 2, 3))
    kz = np.fft.fftfreq(n[2]) * n[2]
    ky = np.fft.fftfreq(n[1]) * n[1]
    kx = np.fft.fftfreq(n[0]) * n[0]
    KZ, KY, KX = np.meshgrid(kz, ky, kx, indexing="ij")
    K = np.stack([KX, KY, KZ])
    k2 = (K ** 2).sum(0)
    F *= (k2 <= kmax * kmax)[None]
    k2s = np.where(k2 == 0, 1.0, k2)
    kdotF = (K * F).sum(0)
    F = F - K * kdotF[None] / k2s[None]
    F[:, 0, 0, 0] = 0.0
    u = np.real(np.fft.ifftn(F, axes=(1, 2, 3)))
    u *= rms / np.sqrt((u ** 2).mean())
    return u


def block_centre_markers(blocks):
    """Particles (float32 [k^3, 3]) at the centres of the level-0 blocks b x b x b, b in `blocks`."""
    c = [8.0 * b + 4.0 for b in blocks]
    pts = [(x, y, z) for z in c for y in c for x in c]
    return np.ascontiguousarray(np.array(pts, dtype=np.float32))


def velocity_moments(level, keys, u_dense):
    """Moments (rho = 1, u sampled from the dense fine field [3, Z, Y, X] at every node's
    fine position, S = u u) of the given blocks: [nb, 10, 512] float64."""
    u = sample_dense(level, keys, u_dense)
    nb = u.shape[0]
    return moments_from_fields(np.zeros((nb, 512)), [u[:, 0], u[:, 1], u[:, 2]])


def unit_directions(n, seeds, kmax=6.0):
    """Divergence-free directions with the spectrum of smooth_random_velocity, each of
    unit L2 norm over all 3 n^3 components: [len(seeds), 3, Z, Y, X] float64."""
    out = []
    for s in seeds:
        d = smooth_random_velocity(n, s, kmax=kmax, rms=1.0)
        out.append(d / np.linalg.norm(d))
    return np.stack(out)


# --- the five workloads ------------------------------------------------------
def workload(name):
    """Static description of a named workload (sizes, boundaries, parameters)."""
    P = PERIODIC
    if name == "tgv64":
        return dict(levels=1, n=(64, 64, 64), bc=(P,) * 6, tau0=0.6, steps=50, amp=0.05)
    if name == "sphere128":
        return dict(levels=2, n=(128, 128, 128), bc=(INFLOW, OUTFLOW, P, P, P, P), uin=(0.05, 0.0, 0.0),
                    tau0=0.6, steps=500, sphere=((64.0, 64.0, 64.0), 12.0))
    if name == "slab512":
        return dict(levels=3, n=(512, 512, 512), bc=(P,) * 6, tau0=0.6, steps=200, amp=0.05,
                    particles=2_000_000, seed=3, lo=(64.0, 64.0, 352.0), hi=(448.0, 448.0, 384.0),
                    v_fine=(0.0, 0.0, -0.02))
    if name == "adjoint128":
        # level 0 over [32, 96)^3: the two-level block set of the sphere case, fixed by
        # eight marker particles at the centres of the level-0 blocks 7..8 per axis
        return dict(levels=2, n=(128, 128, 128), bc=(P,) * 6, tau0=0.6, steps=200, seed=5,
                    kmax=6.0, rms=0.03, box=((48, 48, 48), (80, 80, 80)), checkpoint_every=20,
                    markers=block_centre_markers((7, 8)), direction_seeds=tuple(range(5000, 5016)))
    raise KeyError(name)
