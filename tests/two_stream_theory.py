"""The relativistic two-stream instability (Sec. 5.1.1): its linear theory
(eq. two_stream_dispersion), a seeded setup of two cold counter-streaming
electron beams on a periodic 2D box a few cells across, and the measurement
of the growth rate of a Fourier mode of E_x in its linear stage.  Used to
validate the whole loop (particle step, field solver) of the reference and
of the GPU library against the theory."""
import numpy as np


def two_stream_growth(k, wp, ub):
    """Largest imaginary part of the roots w of
    1 - wp^2/(2 gb^3) [1/(w - k vb)^2 + 1/(w + k vb)^2] = 0 at k."""
    gb = np.sqrt(1 + ub * ub)
    vb = ub / gb
    a = wp * wp / (2 * gb ** 3)
    # (w - kv)^2 (w + kv)^2 - a [(w + kv)^2 + (w - kv)^2] = 0, a quartic in w
    kv = k * vb
    p = np.poly1d([1.0, 0.0, -2 * kv * kv, 0.0, kv ** 4])
    q = np.poly1d([2 * a, 0.0, 2 * a * kv * kv])
    roots = np.roots((p - q).coeffs)
    return float(np.max(roots.imag))


def setup(nx=256, ny=4, ppc=64, wp=0.1, ub=0.5, mode=5, amp=1e-3, temp=1e-4, seed=2511,
          coupling=4 * np.pi):
    """Two beams of electrons (q = -1, m = 1), ppc/2 each per cell, drifting
    along +-x with four-velocity ub, thermal spread sqrt(temp), positions
    displaced by amp * sin(2 pi mode x / nx) to seed one mode; weights such
    that wp^2 = coupling * (weight per unit volume of all electrons).
    Returns (grid dict, species list)."""
    rng = np.random.default_rng(seed)
    ncell = nx * ny
    N = ncell * ppc // 2
    w = wp * wp / coupling / ppc
    cells = np.repeat(np.arange(ncell), ppc // 2)
    species = []
    for sgn in (+1.0, -1.0):
        offs = np.concatenate([rng.random((N, 2)), np.zeros((N, 1))], 1)
        x = cells % nx + offs[:, 0]
        x = np.mod(x + amp * np.sin(2 * np.pi * mode * x / nx), nx)
        cx = np.floor(x).astype(np.int32)
        offs[:, 0] = x - cx
        offs[:, 0] = np.where(offs[:, 0] >= 1.0, 0.0, offs[:, 0])
        cell = np.stack([cx, cells // nx, np.zeros(N, int)], 1).astype(np.int32)
        u = rng.normal(scale=np.sqrt(temp), size=(N, 3))
        u[:, 0] += sgn * ub
        species.append(dict(q=-1.0, m=1.0, cell=cell, offs=offs, u=u, w=np.full(N, w), phi=None,
                            alive=np.ones(N, np.int32)))
    grid = dict(n=(nx, ny, 1), lo=(0.0, 0.0, 0.0), hi=(float(nx), float(ny), 1.0))
    return grid, species


def mode_power(profiles, mode):
    """|FFT|^2 of E_x profiles (times x nx) at one mode, floored at the
    smallest normal double (the fields start at zero, and the log is taken)."""
    p = np.abs(np.fft.rfft(np.asarray(profiles), axis=1)[:, mode]) ** 2
    return np.maximum(p, np.finfo(np.float64).tiny)


def linear_stage_rate(t, log_power):
    """Growth rate of the amplitude (half the slope of ln power against t) in
    the linear stage: a window 6 units long that ends 3 units before the
    first maximum of the smoothed series after t = 5 (earlier, the seeded
    perturbation's other roots have not died out; later, the beams trap)."""
    lp = np.asarray(log_power)
    sm = np.convolve(lp, np.ones(5) / 5, mode="same")
    i1 = int(np.searchsorted(t, 5.0))
    while i1 + 1 < len(sm) - 2 and sm[i1 + 1] >= sm[i1]:
        i1 += 1
    t1 = t[i1]
    sel = (t >= t1 - 9) & (t <= t1 - 3)
    return np.polyfit(t[sel], lp[sel], 1)[0] / 2, (float(t[sel][0]), float(t[sel][-1]))
