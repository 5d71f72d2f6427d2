"""x-z Fourier representation with 3/2 zero padding (oracle; test infrastructure).

Paper: Sec. 2 -- periodic x and z with k_x = 2 pi n / L_x, k_z = 2 pi m / L_z;
Sec. 3.2 -- pseudo-spectral products are de-aliased with the 2/3 rule (the top
third of the harmonics is discarded), and only half of the conjugate-symmetric
harmonic pairs is stored and solved (Appendix A, Hermitian half spectrum).

Conventions (the paper fixes neither sign nor normalisation):
* kept modes: n_x = 0..Nx/2-1 (Nyquist dropped) and |n_z| <= Nz/2-1;
* stored spectral arrays have shape (..., Nx/2, Nz-1) with the z index in FFT
  order: iz = 0..Nz/2-1 is n_z = iz, iz = Nz/2..Nz-2 is n_z = iz - (Nz-1);
* forward transform  f_hat(k) = 1/(Mx Mz) sum_x f(x) exp(-i(kx x + kz z)),
  inverse            f(x)     = sum_k f_hat(k) exp(+i(kx x + kz z)) over the
  full (Hermitian-extended) spectrum, so f_hat(0, 0) is the plane mean;
* physical grid Mx = 3Nx/2, Mz = 3Nz/2 points (3/2 rule == 2/3 truncation);
* the inverse transform uses only the real part of the z-transformed n_x = 0
  column (standard c2r convention), i.e. it implicitly projects that column
  onto its Hermitian part.
"""

import numpy as np


class SpectralGrid:
    """Wavenumbers and de-aliased transforms for one (Lx, Lz, Nx, Nz) box."""

    def __init__(self, Lx, Lz, Nx, Nz):
        if Nx % 2 or Nz % 2:
            raise ValueError("Nx and Nz must be even")
        self.Lx, self.Lz, self.Nx, self.Nz = float(Lx), float(Lz), Nx, Nz
        self.L = Nx // 2            # stored kx columns
        self.P = Nz // 2            # positive kz count (incl. 0)
        self.NZ = Nz - 1            # stored kz entries
        self.Mx = 3 * Nx // 2
        self.Mz = 3 * Nz // 2
        self.nx = np.arange(self.L)
        iz = np.arange(self.NZ)
        self.nz = np.where(iz < self.P, iz, iz - self.NZ)
        self.kx = 2.0 * np.pi * self.nx / self.Lx          # (L,)
        self.kz = 2.0 * np.pi * self.nz / self.Lz          # (NZ,)
        self.KX = self.kx[:, None] * np.ones(self.NZ)[None, :]   # (L, NZ)
        self.KZ = np.ones(self.L)[:, None] * self.kz[None, :]
        self.K2 = self.KX ** 2 + self.KZ ** 2
        # Parseval weight of a stored mode: n_x = 0 once, n_x > 0 twice (+ its conjugate)
        self.mk = np.where(self.nx[:, None] == 0, 1.0, 2.0) * np.ones(self.NZ)[None, :]
        # index of the mode (0, -n_z) for each stored n_x = 0 entry
        self.conj_iz = np.where(self.nz > 0, self.NZ - self.nz,
                                np.where(self.nz < 0, -self.nz, 0))

    # ---- transforms ---------------------------------------------------------
    def to_physical(self, fhat):
        """Inverse transform of stored modes (..., L, NZ) -> real (..., Mz, Mx)."""
        shp = fhat.shape[:-2]
        pad = np.zeros(shp + (self.Mz, self.Mx // 2 + 1), dtype=complex)
        pos = self.nz >= 0
        # rows are z wavenumbers (mod Mz), columns are x wavenumbers 0..L-1
        pad[..., self.nz[pos] % self.Mz, :self.L] = np.swapaxes(fhat[..., :, pos], -1, -2)
        neg = ~pos
        pad[..., self.nz[neg] % self.Mz, :self.L] = np.swapaxes(fhat[..., :, neg], -1, -2)
        return np.fft.irfft2(pad, s=(self.Mz, self.Mx), axes=(-2, -1)) * (self.Mx * self.Mz)

    def to_spectral(self, f):
        """Forward transform real (..., Mz, Mx) -> kept modes (..., L, NZ)."""
        F = np.fft.rfft2(f, axes=(-2, -1)) / (self.Mx * self.Mz)
        rows = self.nz % self.Mz
        sel = F[..., rows, :self.L]                      # (..., NZ, L)
        return np.swapaxes(sel, -1, -2).copy()

    def hermitian_project(self, fhat):
        """Average the n_x = 0 column with its conjugate mirror (n_z <-> -n_z).

        The paper solves only half of the conjugate pairs; the stored n_x = 0
        column holds both n_z and -n_z, which must stay complex conjugates.
        """
        out = fhat.copy()
        col = fhat[..., 0, :]
        mirrored = np.conj(col[..., self.conj_iz])
        out[..., 0, :] = 0.5 * (col + mirrored)
        return out

    def physical_coords(self):
        x = np.arange(self.Mx) * self.Lx / self.Mx
        z = np.arange(self.Mz) * self.Lz / self.Mz
        return x, z
