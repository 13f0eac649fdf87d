"""FP64 oracle of the image-reconstruction use of askadam (paper §2.6.4,
Eq. 7): multi-coil, multi-echo SENSE-type reconstruction with an undersampling
mask, L1 or L2 data loss and an optional 2D total-variation term.

TEST INFRASTRUCTURE ONLY: the tests and the bench's CPU baseline may use this
module; the product path never does.  numpy's FFT is the one library step
(a 2D discrete Fourier transform, unitary normalisation).

Readings (where the paper is silent):
  * operator: k_ec = M_e . F2(C_c . I_e), F2 the unitary 2D DFT over the two
    phase-encoding axes (the paper transforms the read-out axis first and
    reconstructs slice by slice), M_e the sampling mask of echo e, C_c the
    sensitivity of coil c; the paper's inverse-transform notation is the
    same operator up to the sign convention of the exponent;
  * data term: mean over the measured real components,
      D = 1/Nk sum_{e,c, (y,z) in M_e} l(A(I) - k),  Nk = 2 Nc sum_e |M_e|,
    l = |Re r|^2 + |Im r|^2 (L2) or |Re r| + |Im r| (L1);
  * TV (Eq. 7, 2D): anisotropic L1 of the forward differences along y and z
    of the real and of the imaginary part of every echo image, scaled by
    lambda / Npix, Npix = E Ny Nz;
  * the unknowns are Re I and Im I, unbounded (no projection), start 0;
  * Adam, SGDM and RMSProp as for the parameter fits (FP64 here), learning
    rate in image units.
"""
from __future__ import annotations

import numpy as np


def forward(img, coils):
    """img [E, Ny, Nz], coils [Nc, Ny, Nz] complex -> [E, Nc, Ny, Nz] = F2(C_c I_e)."""
    return np.fft.fft2(coils[None, :, :, :] * img[:, None, :, :], norm="ortho")


def adjoint(r, coils):
    """r [E, Nc, Ny, Nz] -> [E, Ny, Nz] = sum_c conj(C_c) F2^H(r_ec)."""
    return (np.conj(coils)[None] * np.fft.ifft2(r, norm="ortho")).sum(axis=1)


def tv2(x):
    """Anisotropic 2D TV of real maps x [E, Ny, Nz] and its subgradient (sign(0) = 0)."""
    R = 0.0
    g = np.zeros_like(x)
    for ax in (1, 2):
        d = np.diff(x, axis=ax)
        R += np.abs(d).sum()
        s = np.sign(d)
        sl_lo = [slice(None)] * 3
        sl_hi = [slice(None)] * 3
        sl_lo[ax] = slice(0, -1)
        sl_hi[ax] = slice(1, None)
        g[tuple(sl_hi)] += s
        g[tuple(sl_lo)] -= s
    return R, g


def loss_grad(img, coils, mask, k, loss=2, lam=0.0):
    """Loss L(I) and its gradient dL/dRe + i dL/dIm, [E, Ny, Nz] complex."""
    E, Nc = k.shape[0], k.shape[1]
    Nk = 2.0 * Nc * mask.sum()
    r = (forward(img, coils) - k) * mask[:, None]
    if loss == 2:
        D = (r.real ** 2 + r.imag ** 2).sum() / Nk
        g = 2.0 * adjoint(r, coils) / Nk
    else:
        D = (np.abs(r.real) + np.abs(r.imag)).sum() / Nk
        s = (np.sign(r.real) + 1j * np.sign(r.imag)) * mask[:, None]
        g = adjoint(s, coils) / Nk
    L = D
    if lam:
        npix = img.size
        Rr, gr = tv2(img.real)
        Ri, gi = tv2(img.imag)
        L += lam / npix * (Rr + Ri)
        g = g + lam / npix * (gr + 1j * gi)
    return L, g


def recon(k, coils, mask, n_iter=100, lr=0.01, loss=2, lam=0.0, beta1=0.9, beta2=0.999,
          eps=1e-8, init=None, optimizer="adam", momentum=0.9, rho=0.9):
    """askadam on Re I and Im I from I = 0 (or init); returns (image, loss history).

    optimizer "adam" | "sgdm" | "rmsprop", with the update rules of the
    parameter fits: SGDM vel = momentum vel - lr g, I += vel; RMSProp
    v = rho v + (1 - rho) g^2, I -= lr g / (sqrt(v) + eps)."""
    E, Ny, Nz = mask.shape
    img = np.zeros((E, Ny, Nz), complex) if init is None else np.array(init, complex)
    m = np.zeros((2, E, Ny, Nz))
    v = np.zeros((2, E, Ny, Nz))
    hist = []
    for t in range(1, n_iter + 1):
        L, g = loss_grad(img, coils, mask, k, loss, lam)
        hist.append(L)
        gg = np.stack([g.real, g.imag])
        if optimizer == "adam":
            m = beta1 * m + (1 - beta1) * gg
            v = beta2 * v + (1 - beta2) * gg * gg
            c1 = 1.0 / (1.0 - beta1 ** t)
            c2 = 1.0 / (1.0 - beta2 ** t)
            step = lr * (m * c1) / (np.sqrt(v * c2) + eps)
        elif optimizer == "sgdm":
            m = momentum * m - lr * gg
            step = -m
        elif optimizer == "rmsprop":
            v = rho * v + (1 - rho) * gg * gg
            step = lr * gg / (np.sqrt(v) + eps)
        else:
            raise ValueError(optimizer)
        img = (img.real - step[0]) + 1j * (img.imag - step[1])
    return img, np.array(hist)
