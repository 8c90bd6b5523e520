"""Eq. (2): H(r0) = -sum_r N(r - r0) M(r) over all cells of the mesh.

* ``demag_direct``: the sum as written, O(N^2), for tiny meshes.  It is the
  plain definition and is the pin for ``demag_fft``.
* ``demag_fft``: the same sum by the convolution theorem (Sec. II names FFT
  evaluation, ref. [25]).  Each axis of length n > 1 is zero-padded to 2n
  (open boundaries: no periodic images), a length-1 axis is not padded.  N is
  placed at wrap-around indices (offset d at index d mod 2n).  Because every
  component of N is even under r -> -r (diagonal: even in each axis;
  off-diagonal: odd in exactly two axes) the correlation of Eq. (2) equals a
  convolution.

Arrays use the layout (3, nz, ny, nx), x fastest.  ``Nfull`` is the output of
``newell.tensor_full`` (or any tensor of that shape: the two functions only
implement Eq. (2) for the given N).

Pins (tests/test_oracle_demag.py): FFT vs direct sum on tiny meshes; single
cell gives -N00 M; uniform M gives a mesh-mean field of -D_prism M with
Aharoni's whole-box factors; linearity.
"""

import numpy as np
import scipy.fft as sfft

# component index of N_ij in the 6-vector (xx, yy, zz, xy, xz, yz)
_IJ = ((0, 3, 4), (3, 1, 5), (4, 5, 2))


def demag_direct(M, Nfull):
    """Direct O(N^2) evaluation of Eq. (2)."""
    _, nz, ny, nx = M.shape
    H = np.zeros_like(M, dtype=np.float64)
    zs, ys, xs = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    for z0 in range(nz):
        for y0 in range(ny):
            for x0 in range(nx):
                # N(r - r0) for every source cell r
                Nr = Nfull[:, zs - z0 + nz - 1, ys - y0 + ny - 1, xs - x0 + nx - 1]
                for i in range(3):
                    H[i, z0, y0, x0] = -sum(np.sum(Nr[_IJ[i][j]] * M[j]) for j in range(3))
    return H


def padded_shape(n):
    """Zero-padded FFT lengths per axis (nx, ny, nz) -> (Px, Py, Pz): 2n for n > 1, else 1."""
    return tuple(2 * v if v > 1 else 1 for v in n)


def kspace_kernel(Nfull, n):
    """Real-space N placed at wrap-around indices of the padded grid, transformed by rfftn.

    Returns a complex array (6, Pz, Py, Px//2+1).  Its imaginary part is zero
    up to rounding by the parity of N (pinned in tests)."""
    nx, ny, nz = n
    Px, Py, Pz = padded_shape(n)
    K = np.zeros((6, Pz, Py, Px))
    dz = np.arange(-(nz - 1), nz) % Pz
    dy = np.arange(-(ny - 1), ny) % Py
    dx = np.arange(-(nx - 1), nx) % Px
    K[:, dz[:, None, None], dy[None, :, None], dx[None, None, :]] = Nfull
    return sfft.rfftn(K, axes=(1, 2, 3))


def demag_fft(M, Nfull, Khat=None, workers=None):
    """Zero-padded FFT evaluation of Eq. (2)."""
    _, nz, ny, nx = M.shape
    n = (nx, ny, nz)
    Px, Py, Pz = padded_shape(n)
    if Khat is None:
        Khat = kspace_kernel(Nfull, n)
    Mh = sfft.rfftn(M.astype(np.float64), s=(Pz, Py, Px), axes=(1, 2, 3), workers=workers)
    Hh = np.empty_like(Mh)
    for i in range(3):
        Hh[i] = -(Khat[_IJ[i][0]] * Mh[0] + Khat[_IJ[i][1]] * Mh[1] + Khat[_IJ[i][2]] * Mh[2])
    H = sfft.irfftn(Hh, s=(Pz, Py, Px), axes=(1, 2, 3), workers=workers)
    return np.ascontiguousarray(H[:, :nz, :ny, :nx])
