"""Surface quasi-geostrophic (nonlinear Eady) model, pseudo-spectral, FP64 (oracle; test
infrastructure only).

The paper's test model (Sec. II-B) is SQG turbulence of Tulloch & Smith: potential
temperature on two rigid boundaries (ground z = 0 and lid z = 1) of an f-plane layer with
uniform stratification, zero interior potential vorticity and a uniform vertical shear of
the basic flow; FFT-based spatial discretisation with 2/3 dealiasing, RK4 in time and an
implicit treatment of hyperdiffusion.  The paper leaves the parameters to an external code
that is not available here; this module is written from the published physics in
nondimensional units: f = N = H = 1 (lengths in Rossby radii N H / f), total shear
Lambda = 1 (basic flow U(z) = Lambda (z - 1/2)), domain [0, Lx)^2 doubly periodic.

Equations (theta_i on level i, psi_i the boundary streamfunctions):
    d theta_i/dt + (U_i + u_i) d theta_i/dx + v_i (d theta_i/dy - Lambda) = D(theta_i),
    u = -d psi/dy, v = d psi/dx,
with the zero-PV inversion (wavenumber magnitude K):
    psi_0 = -theta_0 / (K tanh K) + theta_1 / (K sinh K)
    psi_1 = -theta_0 / (K sinh K) + theta_1 / (K tanh K)
and D a hyperdiffusion of order 2p plus a thermal relaxation toward the basic state with
time scale tau (which lets the turbulence equilibrate), both linear and applied exactly
over each step:
    theta_hat <- theta_hat * exp(-dt * nu * (K / K_max)^(2p) - dt / tau).
State layout: (2, n, n) float64, level-major (component e = level*n*n + iy*n + ix).
"""
import numpy as np


class SQG:
    def __init__(self, n=128, lx=20.0, shear=1.0, dt=0.025, diff_order=8, diff_efold=None,
                 dealias=True, relax_time=np.inf):
        self.n, self.lx, self.shear, self.dt = n, lx, shear, dt
        k1 = 2.0 * np.pi / lx
        kx = np.fft.rfftfreq(n, 1.0 / n) * k1
        ky = np.fft.fftfreq(n, 1.0 / n) * k1
        self.kx = kx[None, :]
        self.ky = ky[:, None]
        K = np.sqrt(self.kx ** 2 + self.ky ** 2)
        Ks = np.where(K > 0, K, 1.0)
        inv_tanh = np.where(K > 0, 1.0 / (Ks * np.tanh(Ks)), 0.0)
        inv_sinh = np.where(K > 0, 1.0 / (Ks * np.sinh(Ks)), 0.0)
        self.inv_tanh, self.inv_sinh = inv_tanh, inv_sinh
        kmax = k1 * (n // 2)
        # 2/3 rule on both wavenumber components
        self.mask = ((np.abs(np.fft.fftfreq(n, 1.0 / n))[:, None] < n / 3.0) &
                     (np.abs(np.fft.rfftfreq(n, 1.0 / n))[None, :] < n / 3.0)) if dealias else 1.0
        # the highest retained wavenumber is damped with an e-folding time of diff_efold
        efold = diff_efold if diff_efold is not None else 10.0 * dt
        self.hyper = (np.exp(-dt / efold * (K / (2.0 / 3.0 * kmax)) ** diff_order)
                      if diff_efold != np.inf else np.ones_like(K))
        # thermal relaxation of theta toward the basic state (linear damping, exact per step)
        self.hyper = self.hyper * np.exp(-dt / relax_time)
        self.U = np.array([-0.5 * shear, 0.5 * shear])

    # spectral helpers ---------------------------------------------------------------
    def fft(self, f):
        return np.fft.rfft2(f, axes=(-2, -1))

    def ifft(self, fh):
        return np.fft.irfft2(fh, s=(self.n, self.n), axes=(-2, -1))

    def invert(self, th):
        """Boundary streamfunctions from boundary temperatures (spectral, (..., 2, n, n/2+1))."""
        t0, t1 = th[..., 0, :, :], th[..., 1, :, :]
        p0 = -t0 * self.inv_tanh + t1 * self.inv_sinh
        p1 = -t0 * self.inv_sinh + t1 * self.inv_tanh
        return np.stack([p0, p1], axis=-3)

    def tendency(self, th):
        """d theta_hat / dt without diffusion (spectral in, spectral out)."""
        ps = self.invert(th)
        ik, il = 1j * self.kx, 1j * self.ky
        u = self.ifft(-il * ps)
        v = self.ifft(ik * ps)
        tx = self.ifft(ik * th)
        ty = self.ifft(il * th)
        U = self.U.reshape((1,) * (th.ndim - 3) + (2, 1, 1))
        adv = (U + u) * tx + v * (ty - self.shear)
        return -self.fft(adv) * self.mask

    def step_spectral(self, th):
        dt = self.dt
        k1 = self.tendency(th)
        k2 = self.tendency(th + 0.5 * dt * k1)
        k3 = self.tendency(th + 0.5 * dt * k2)
        k4 = self.tendency(th + dt * k3)
        return (th + dt / 6.0 * (k1 + 2 * k2 + 2 * k3 + k4)) * self.hyper

    def run(self, theta, n_steps):
        """Advance physical states (..., 2, n, n) by n_steps steps."""
        th = self.fft(np.asarray(theta, dtype=np.float64)) * self.mask
        for _ in range(n_steps):
            th = self.step_spectral(th)
        return self.ifft(th)


def eady_growth_rate(k, K, shear=1.0):
    """Textbook Eady growth rate (f = N = H = 1) of a mode with zonal wavenumber k and total
    wavenumber K: sigma = (k shear / K) sqrt((coth(K/2) - K/2)(K/2 - tanh(K/2))), zero when
    the product is negative (short-wave cutoff)."""
    h = 0.5 * K
    prod = (1.0 / np.tanh(h) - h) * (h - np.tanh(h))
    return np.where(prod > 0, k * shear / K * np.sqrt(np.maximum(prod, 0.0)), 0.0)
