"""Algorithmic work and traffic of each kernel, per unit and per launch.

These are the models against which the roofline fractions are reported; each
states the minimum bytes (or flops) the kernel's schedule must move (or do),
not what caches happen to save.

Units:
  stencil step   cell-update = one grid cell of the padded grid advanced one
                 time step for one Green function
  DFT chunk      sample-frequency = one subgrid sample entering one
                 frequency's accumulator
  Hessian        complex multiply-add of the contraction (upper triangle)
"""
from __future__ import annotations


def padded_cells(nz, nx, nb):
    return (nz + 2 * nb) * (nx + 2 * nb)


def subgrid_points(nz, nx, stride):
    return ((nz + stride - 1) // stride) * ((nx + stride - 1) // stride)


def stencil_bytes_per_cell_update(nz, nx, nb, stride, nrb, tblock):
    """Marching step of tblock levels: u and w read once and written once per
    launch (16 B per cell), the coefficient plane read once per launch and
    shared by the nrb receivers (4 B per cell), and every level's subgrid sample
    (4 B) written to the staging buffer."""
    cells = padded_cells(nz, nx, nb)
    sub = subgrid_points(nz, nx, stride)
    return (16.0 + 4.0 / nrb) / tblock + 4.0 * sub / cells


def stencil_cell_updates_per_survey(nz, nx, nb, nr, nt):
    return padded_cells(nz, nx, nb) * nr * (nt - 1)


def dft_bytes_per_survey(nz, nx, stride, nr, nt, nf, chunk):
    """Staged samples read once (4 B each) and the complex64 accumulators read
    and written once per chunk."""
    sub = subgrid_points(nz, nx, stride)
    nchunk = -(-nt // chunk)
    return 4.0 * sub * nr * nt + 16.0 * sub * nr * nf * nchunk


def dft_flops_per_survey(nz, nx, stride, nr, nt, nf):
    """4 real flops (2 FMAs) per sample-frequency, real sample x complex twiddle."""
    return 4.0 * subgrid_points(nz, nx, stride) * nr * nt * nf


def herk_flops_per_survey(nz, nx, stride, nr, nf):
    """Upper triangle incl. diagonal of the complex contraction, 8 flops per
    complex multiply-add."""
    return 8.0 * nr * (nr + 1) / 2 * subgrid_points(nz, nx, stride) * nf


def herk_bf16_mfma_flops_per_survey(nr, nsub, nf, tile=64):
    """BF16 MFMA flops the split contraction executes: 16 real products of
    K = nsub (hi/lo x hi/lo for Re and Im) on every tile x tile block on or
    above the block diagonal (64 x 64 tile pairs, or the 32 x 32 block pairs of
    the whole-matrix form)."""
    nb = -(-nr // tile)
    pairs = nb * (nb + 1) // 2
    return 2.0 * 16 * pairs * tile * tile * nsub * nf


def herk_bytes_per_survey(nz, nx, stride, nr, nf):
    """Reading the complex64 spectra once."""
    return 8.0 * subgrid_points(nz, nx, stride) * nr * nf
