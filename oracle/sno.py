"""Learned spin-up: channel form of a flow state and a spectral neural operator.

TEST INFRASTRUCTURE ONLY (see the package docstring): plain FP64 numpy, written
for clarity.  The paper starts every ensemble member from a perturbed state and
lets the DNS run through the transient to turbulence; the learned spin-up
replaces most of that transient by a few applications of a small spectral
neural operator (a Fourier neural operator acting on x-z planes), after which
the plain DNS continues and checks every member.

Channel form of a state (one member):
  * u, v, w on the 3/2-padded x-z grid (Mx x Mz points, as used for the
    advection term, Sec. 3.2) at every Chebyshev node y_j (Sec. 2);
  * along y, each field is replaced by the coefficients a_k, k < My, of its
    Chebyshev interpolant f(y) = sum_k a_k T_k(y) through the My nodes;
  * channel index c = field * My + k (field 0, 1, 2 = u, v, w), point index
    p = iz * Mx + ix; array shape (members, 3 My, Mz Mx).
The inverse map rebuilds an admissible state: v at the interior nodes, eta =
i kz u - i kx w (the wall-normal vorticity, Sec. 2), U00 and W00 from the (0, 0)
modes with the wall values of the boundary conditions, the n_x = 0 column made
Hermitian.  Velocities recovered from (v, eta) then satisfy continuity and the
no-slip conditions exactly (Sec. 3.2, u/w recovery), whatever the channels.

Spectral neural operator (width W, n_layers layers, retained modes mx x mz):
  h_0 = W_lift x + b_lift                               (pointwise, C -> W)
  h_l = GELU(W_l h_{l-1} + b_l + S_l h_{l-1}),  l = 1..n_layers
  S h = IDFT( R[m] DFT(h)[m] ) over retained modes m (complex W x W per mode)
  y   = x + Q h_L + b_Q                                 (pointwise, W -> C)
  DFT: X[m] = 1/(Mx Mz) sum_p h[p] exp(-i theta_m(p)),
       theta_m(p) = 2 pi (kx ix / Mx + kz iz / Mz),
       kx = 0..mx-1, kz = q for q < mz/2 else q - mz (q = 0..mz-1), m = kx mz + q;
  IDFT: g[p] = sum_m w_kx Re(Y[m] exp(+i theta_m(p))), w_0 = 1, w_kx>0 = 2.
  GELU(z) = z Phi(z) (Phi the standard normal CDF).
  Loss: mean over samples of ||y_hat - y||_2 / ||y||_2.  Optimiser: AdamW.
Parameter vector (flat, in this order): W_lift (W x C), b_lift (W); per layer
W_l (W x W), b_l (W), Re R_l (M x W x W), Im R_l (M x W x W); Q (C x W), b_Q (C),
with R[m][o][i] mapping input channel i to output channel o.
"""

import numpy as np
from scipy.special import erf

from .cheb import nodes


# ---- channel form ---------------------------------------------------------------
def chebyshev_vandermonde(My):
    """T[j][k] = T_k(y_j) on the ascending Gauss-Lobatto nodes."""
    y = nodes(My)
    return np.cos(np.arange(My)[None, :] * np.arccos(np.clip(y, -1.0, 1.0))[:, None])


def channels_from_state(sim, v, eta, U, W):
    """State (the DNS layout) -> channel form (E, 3 My, Mz Mx) in FP64."""
    g = sim.grid
    vel = sim.velocities(v, eta, U, W)
    T = chebyshev_vandermonde(sim.My)
    out = []
    for f in ("u", "v", "w"):
        phys = g.to_physical(vel[f])                       # (E, My, Mz, Mx)
        coef = np.linalg.solve(T, phys.reshape(phys.shape[0], sim.My, -1))  # per member
        out.append(coef)
    return np.concatenate(out, axis=1)


def state_from_channels(sim, ch):
    """Channel form -> admissible state (v, eta, U, W) in the DNS layout."""
    g = sim.grid
    E = ch.shape[0]
    My, N = sim.My, sim.N
    T = chebyshev_vandermonde(My)
    spec = []
    for f in range(3):
        vals = np.einsum("jk,ekp->ejp", T, ch[:, f * My:(f + 1) * My])
        phys = vals.reshape(E, My, g.Mz, g.Mx)
        spec.append(g.to_spectral(phys))                  # (E, My, L, NZ)
    uh, vh, wh = spec
    v = np.moveaxis(vh[:, 1:-1], 1, -1).copy()             # (E, L, NZ, N)
    eta_full = 1j * g.KZ * uh - 1j * g.KX * wh
    eta = np.moveaxis(eta_full[:, 1:-1], 1, -1).copy()
    v[:, 0, 0, :] = 0.0
    eta[:, 0, 0, :] = 0.0
    v = np.moveaxis(g.hermitian_project(np.moveaxis(v, -1, 1)), 1, -1)
    eta = np.moveaxis(g.hermitian_project(np.moveaxis(eta, -1, 1)), 1, -1)
    Ufull = uh[:, :, 0, 0].real.copy()
    Wfull = wh[:, :, 0, 0].real.copy()
    lam = sim.laminar_profile()
    Ufull[:, 0], Ufull[:, -1] = lam[0], lam[-1]
    Wfull[:, 0], Wfull[:, -1] = 0.0, 0.0
    del N
    return v, eta, Ufull, Wfull


# ---- spectral neural operator --------------------------------------------------------
def mode_wavenumbers(mx, mz):
    kx = np.repeat(np.arange(mx), mz)
    q = np.tile(np.arange(mz), mx)
    kz = np.where(q < mz // 2, q, q - mz)
    return kx, kz


def dft_matrices(Mx, Mz, mx, mz):
    """Dense real matrices of the truncated DFT and its inverse.

    D (P x 2M): [Re X | Im X] = h @ D;  Dinv (2M x P): g = [Re Y | Im Y] @ Dinv.
    """
    kx, kz = mode_wavenumbers(mx, mz)
    iz, ix = np.divmod(np.arange(Mz * Mx), Mx)
    theta = 2.0 * np.pi * (np.outer(ix, kx) / Mx + np.outer(iz, kz) / Mz)   # (P, M)
    D = np.concatenate([np.cos(theta), -np.sin(theta)], axis=1) / (Mx * Mz)
    w = np.where(kx == 0, 1.0, 2.0)
    Dinv = np.concatenate([w[:, None] * np.cos(theta).T, -w[:, None] * np.sin(theta).T], axis=0)
    return D, Dinv


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / np.sqrt(2.0)))


def gelu_grad(z):
    return 0.5 * (1.0 + erf(z / np.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / np.sqrt(2.0 * np.pi)


class SNOConfig:
    def __init__(self, channels, width, layers, Mx, Mz, mx, mz):
        self.C, self.W, self.L = channels, width, layers
        self.Mx, self.Mz, self.mx, self.mz = Mx, Mz, mx, mz
        self.M = mx * mz
        self.P = Mx * Mz

    def shapes(self):
        C, W, M = self.C, self.W, self.M
        s = [("lift_w", (W, C)), ("lift_b", (W,))]
        for l in range(self.L):
            s += [(f"w{l}", (W, W)), (f"b{l}", (W,)), (f"rr{l}", (M, W, W)), (f"ri{l}", (M, W, W))]
        s += [("q_w", (C, W)), ("q_b", (C,))]
        return s

    def num_params(self):
        return int(sum(np.prod(sh) for _, sh in self.shapes()))

    def unpack(self, theta):
        out, o = {}, 0
        for name, sh in self.shapes():
            n = int(np.prod(sh))
            out[name] = theta[o:o + n].reshape(sh)
            o += n
        return out

    def pack(self, parts):
        return np.concatenate([np.asarray(parts[name], dtype=float).ravel() for name, _ in self.shapes()])


def spectral_mix(rr, ri, Xh, M):
    """Y[b,o,m] = sum_i R[m,o,i] X[b,i,m] (complex), in the real layout [Re | Im]."""
    Xr, Xi = Xh[..., :M], Xh[..., M:]
    Yr = np.einsum("moi,bim->bom", rr, Xr) - np.einsum("moi,bim->bom", ri, Xi)
    Yi = np.einsum("moi,bim->bom", ri, Xr) + np.einsum("moi,bim->bom", rr, Xi)
    return np.concatenate([Yr, Yi], axis=-1)


def forward(cfg, theta, x):
    """y_hat for x (B, C, P); returns (y_hat, cache for backward)."""
    p = cfg.unpack(theta)
    D, Dinv = dft_matrices(cfg.Mx, cfg.Mz, cfg.mx, cfg.mz)
    h = np.einsum("oi,bip->bop", p["lift_w"], x) + p["lift_b"][None, :, None]
    cache = {"x": x, "h": [h], "z": [], "xh": [], "D": D, "Dinv": Dinv}
    for l in range(cfg.L):
        xh = h @ D                                          # (B, W, 2M)
        yh = spectral_mix(p[f"rr{l}"], p[f"ri{l}"], xh, cfg.M)
        z = np.einsum("oi,bip->bop", p[f"w{l}"], h) + p[f"b{l}"][None, :, None] + yh @ Dinv
        h = gelu(z)
        cache["xh"].append(xh)
        cache["z"].append(z)
        cache["h"].append(h)
    y = x + np.einsum("ci,bip->bcp", p["q_w"], h) + p["q_b"][None, :, None]
    return y, cache


def rel_l2_loss(yhat, y):
    """Mean over samples of ||yhat - y|| / ||y||, and its gradient in yhat."""
    B = y.shape[0]
    d = (yhat - y).reshape(B, -1)
    nd = np.linalg.norm(d, axis=1)
    ny = np.linalg.norm(y.reshape(B, -1), axis=1)
    loss = float(np.mean(nd / ny))
    scale = np.where(nd > 0, 1.0 / (np.where(nd > 0, nd, 1.0) * ny * B), 0.0)
    return loss, (d * scale[:, None]).reshape(y.shape)


def backward(cfg, theta, cache, dy):
    """Gradient of a scalar loss with respect to theta, given dL/dy_hat."""
    p = cfg.unpack(theta)
    D, Dinv, x = cache["D"], cache["Dinv"], cache["x"]
    M = cfg.M
    g = {}
    h_last = cache["h"][-1]
    g["q_w"] = np.einsum("bcp,bip->ci", dy, h_last)
    g["q_b"] = dy.sum(axis=(0, 2))
    dh = np.einsum("ci,bcp->bip", p["q_w"], dy)
    for l in reversed(range(cfg.L)):
        z, h_prev, xh = cache["z"][l], cache["h"][l], cache["xh"][l]
        dz = dh * gelu_grad(z)
        g[f"b{l}"] = dz.sum(axis=(0, 2))
        g[f"w{l}"] = np.einsum("bop,bip->oi", dz, h_prev)
        dh = np.einsum("oi,bop->bip", p[f"w{l}"], dz)
        dyh = dz @ Dinv.T                                   # (B, W, 2M)
        dYr, dYi = dyh[..., :M], dyh[..., M:]
        Xr, Xi = xh[..., :M], xh[..., M:]
        g[f"rr{l}"] = np.einsum("bom,bim->moi", dYr, Xr) + np.einsum("bom,bim->moi", dYi, Xi)
        g[f"ri{l}"] = -np.einsum("bom,bim->moi", dYr, Xi) + np.einsum("bom,bim->moi", dYi, Xr)
        rr, ri = p[f"rr{l}"], p[f"ri{l}"]
        dXr = np.einsum("moi,bom->bim", rr, dYr) + np.einsum("moi,bom->bim", ri, dYi)
        dXi = -np.einsum("moi,bom->bim", ri, dYr) + np.einsum("moi,bom->bim", rr, dYi)
        dh = dh + np.concatenate([dXr, dXi], axis=-1) @ D.T
    g["lift_w"] = np.einsum("bop,bip->oi", dh, x)
    g["lift_b"] = dh.sum(axis=(0, 2))
    return cfg.pack(g)


def adamw_step(theta, grad, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8, weight_decay=1e-4):
    """One AdamW update (decoupled weight decay); t is the 1-based step count."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    theta = theta - lr * weight_decay * theta - lr * mhat / (np.sqrt(vhat) + eps)
    return theta, m, v
