"""The oracle's pins catch plausible mistakes: each test plants one mistake in
the oracle (on the CPU, through monkeypatch) and checks that a pin written
against the paper or the mathematics now fails.  Together with the pins
passing on the unmodified oracle, this shows the pins are not vacuous."""
import math

import numpy as np
import pytest

from oracle import bounded, transforms
from oracle import unbounded as ub

import test_oracle_bounded as pb
import test_oracle_kernels as pk
import test_oracle_operators as po
import test_oracle_transforms as pt
import test_oracle_unbounded as pu


def _fails(fn, *args):
    with pytest.raises(AssertionError):
        fn(*args)


def test_eigenvalue_index_shift_is_caught(monkeypatch):
    # Table 1, FD2 Dirichlet regular, with k in place of k + 1
    orig = bounded.eigenvalues

    def wrong(bc, grid, operator, n, length, h):
        lam = orig(bc, grid, operator, n, length, h)
        if bc == "dirichlet" and grid == "regular" and operator == "fd2":
            k = np.arange(n, dtype=np.float64)
            lam = -4.0 / (h * h) * np.sin(np.pi * k / (2.0 * (n + 1))) ** 2
        return lam

    monkeypatch.setattr(bounded, "eigenvalues", wrong)
    _fails(pb.test_fd2_matches_dense_solve, "dirichlet", "regular", 2, False)


def test_boundary_weight_sign_is_caught(monkeypatch):
    # Neumann staggered face terms with the sides swapped
    orig = bounded.apply_boundary_values

    def wrong(f, bc, grid, hs, faces):
        if bc == "neumann" and grid == "staggered":
            faces = {(a, 1 - s): g for (a, s), g in faces.items()}
        return orig(f, bc, grid, hs, faces)

    monkeypatch.setattr(bounded, "apply_boundary_values", wrong)
    _fails(pb.test_fd2_matches_dense_solve, "neumann", "staggered", 2, True)


def test_sine_transform_index_is_caught(monkeypatch):
    # DST-II with (j + 1) in place of (2 j + 1) / 2
    def wrong(n):
        k = np.arange(n)[:, None]
        j = np.arange(n)[None, :]
        return 2.0 * np.sin(np.pi * (j + 1) * (k + 1) / n)

    monkeypatch.setitem(transforms.MATRICES, "dst2", wrong)
    _fails(pt.test_matrix_matches_library, "dst2", 8)


def test_missing_cell_volume_is_caught(monkeypatch):
    # the discrete convolution without the quadrature weight prod(H)
    def wrong(shape, hs, sigma, kernel="g2"):
        return np.fft.rfftn(ub.green_extended(shape, hs, sigma, kernel))

    monkeypatch.setattr(ub, "green_spectrum", wrong)
    _fails(pu.test_gaussian_closed_form, 32)


def test_unmirrored_green_function_is_caught(monkeypatch):
    # G laid out as G(m H) on the doubled grid instead of G(min(m, 2n - m) H)
    monkeypatch.setattr(ub, "mirrored_distance", lambda n, h: np.arange(2 * n, dtype=np.float64) * float(h))
    _fails(pu.test_doubling_equals_direct_sum)


def test_wavenumber_sign_is_caught(monkeypatch):
    # negative wavenumbers folded to positive ones (m in place of m - M)
    orig = ub.wavenumbers

    def wrong(shape, hs):
        return [np.abs(k) for k in orig(shape, hs)]

    monkeypatch.setattr(ub, "wavenumbers", wrong)
    _fails(pu.test_gradient_and_curl_closed_form)


def test_hermite_sign_is_caught(monkeypatch):
    # order-4 kernel with the Hermite correction subtracted instead of added
    def wrong(r, sigma, order):
        r = np.asarray(r, dtype=np.float64)
        rho = r / sigma
        from scipy.special import erf
        acc = erf(rho / math.sqrt(2)) - math.sqrt(2 / math.pi) * np.exp(-0.5 * rho * rho) * rho / 2
        return -acc / (4 * np.pi * r)

    monkeypatch.setattr(ub, "green_gauss", wrong)
    _fails(pk.test_gauss_kernel_is_its_spectral_integral, 4)


def test_spectral_cutoff_is_caught(monkeypatch):
    # cutoff at the half-grid wavenumber pi / (2 H)
    orig = ub.green_spectral
    monkeypatch.setattr(ub, "green_spectral", lambda r, h: orig(r, 2 * h))
    _fails(pk.test_spectral_kernel_is_its_spectral_integral)


def test_laplacian_sign_is_caught(monkeypatch):
    # NABLA with the sign of (i k)^2 dropped: negate the outer of the two
    # first-derivative applications
    orig = bounded.periodic_gradient
    calls = {"n": 0}

    def wrong(psi, lengths):
        calls["n"] += 1
        g = orig(psi, lengths)
        return [-x for x in g] if calls["n"] % 2 == 0 else g

    monkeypatch.setattr(bounded, "periodic_gradient", wrong)
    _fails(po.test_periodic_nabla_returns_source)


def test_bounded_derivative_sign_is_caught(monkeypatch):
    # Neumann: d/dx cos taken as +w sin
    orig = bounded.eigenfunctions

    def wrong(bc, n, length, x):
        phi, dphi = orig(bc, n, length, x)
        return (phi, -dphi) if bc == "neumann" else (phi, dphi)

    monkeypatch.setattr(bounded, "eigenfunctions", wrong)
    _fails(pb.test_bounded_gradient_of_eigenmodes, "neumann", "staggered", 2, "ps")


def test_bounded_derivative_chain_factor_is_caught(monkeypatch):
    # Dirichlet: the factor pi (k + 1) / L of the chain rule dropped
    orig = bounded.eigenfunctions

    def wrong(bc, n, length, x):
        phi, dphi = orig(bc, n, length, x)
        if bc == "dirichlet":
            w = np.pi * (np.arange(n) + 1.0) / float(length)
            dphi = dphi / w[None, :]
        return phi, dphi

    monkeypatch.setattr(bounded, "eigenfunctions", wrong)
    _fails(pb.test_bounded_gradient_of_eigenmodes, "dirichlet", "regular", 3, "fd2")


def test_1d_hermite_correction_sign_is_caught(monkeypatch):
    # 1D order-4 kernel with the Hermite correction subtracted instead of added
    orig = ub.green_gauss_1d

    def wrong(x, sigma, order):
        return 2.0 * ub.green_g2_1d(x, sigma) - orig(x, sigma, order)

    monkeypatch.setattr(ub, "green_gauss_1d", wrong)
    _fails(pk.test_1d_gauss_kernel_second_derivative_is_its_source, 4)


def test_periodic_curl_component_swap_is_caught(monkeypatch):
    # u_y and u_z exchanged in the periodic 3D curl
    orig = bounded.periodic_curl

    def wrong(psi, lengths):
        u = orig(psi, lengths)
        return [u[0], u[2], u[1]]

    monkeypatch.setattr(bounded, "periodic_curl", wrong)
    _fails(po.test_periodic_3d_curl_closed_form)


def test_periodic_curl_sign_is_caught(monkeypatch):
    # u_x = d_z psi_y - d_y psi_z (one component with its sign flipped)
    orig = bounded.periodic_curl

    def wrong(psi, lengths):
        u = orig(psi, lengths)
        return [-u[0], u[1], u[2]]

    monkeypatch.setattr(bounded, "periodic_curl", wrong)
    _fails(po.test_periodic_3d_curl_closed_form)


def test_periodic_gradient_axis_is_caught(monkeypatch):
    # the wavenumber of axis 1 used for axis 2 (anisotropic box)
    orig = bounded.periodic_gradient

    def wrong(psi, lengths):
        return orig(psi, [lengths[0], lengths[1], lengths[1]] if len(lengths) == 3 else lengths)

    monkeypatch.setattr(bounded, "periodic_gradient", wrong)
    _fails(po.test_periodic_3d_gradient_closed_form)


def test_bounded_curl_component_swap_is_caught(monkeypatch):
    # Dirichlet / Neumann curl with u_x and u_y exchanged
    orig = bounded.bounded_curl

    def wrong(psi, bc, grid, nc, lengths):
        u = orig(psi, bc, grid, nc, lengths)
        return [u[1], u[0], u[2]]

    monkeypatch.setattr(bounded, "bounded_curl", wrong)
    _fails(pb.test_bounded_curl_and_div_of_eigenmodes, "neumann", "staggered", "ps")


def test_bounded_curl_sign_is_caught(monkeypatch):
    # u_z = d_y psi_x - d_x psi_y (sign of one component flipped)
    orig = bounded.bounded_curl

    def wrong(psi, bc, grid, nc, lengths):
        u = orig(psi, bc, grid, nc, lengths)
        return [u[0], u[1], -u[2]]

    monkeypatch.setattr(bounded, "bounded_curl", wrong)
    _fails(pb.test_bounded_curl_and_div_of_eigenmodes, "dirichlet", "regular", "fd2")


def test_bounded_second_derivative_factor_is_caught(monkeypatch):
    # second derivative of the series with -w in place of -w^2
    orig = bounded.bounded_derivative

    def wrong(psi, bc, grid, nc, lengths, axis, order=1):
        if order != 2:
            return orig(psi, bc, grid, nc, lengths, axis, order)
        d1 = orig(psi, bc, grid, nc, lengths, axis, 2)
        w = np.pi / float(lengths[axis])
        return d1 / w

    monkeypatch.setattr(bounded, "bounded_derivative", wrong)
    _fails(pb.test_bounded_laplacian_of_eigenmodes, "dirichlet", "staggered", 2, "ps")


def test_bounded_divergence_axis_is_caught(monkeypatch):
    # divergence built from d psi_c / d x_(c+1) instead of d psi_c / d x_c
    import oracle
    orig = bounded.bounded_derivative

    def wrong(psi, bc, grid, nc, lengths, axis, order=1):
        return orig(psi, bc, grid, nc, lengths, (axis + 1) % np.ndim(psi), order)

    monkeypatch.setattr(bounded, "bounded_derivative", wrong)
    _fails(pb.test_bounded_curl_and_div_of_eigenmodes, "neumann", "regular", "fd2")


def test_mixed_face_weight_axis_is_caught(monkeypatch):
    # every face weighted by the condition of axis 0
    import test_oracle_mixed as pm
    orig = bounded.apply_boundary_values_mixed

    def wrong(f, bcs, grid, hs, faces):
        return orig(f, [bcs[0]] * len(bcs), grid, hs, faces)

    monkeypatch.setattr(bounded, "apply_boundary_values_mixed", wrong)
    _fails(pm.test_mixed_fd2_matches_dense_solve, ["dirichlet", "neumann"], "staggered", True)


def test_mixed_periodic_eigenvalue_is_caught(monkeypatch):
    # a periodic axis given the Neumann eigenvalues (pi k / L instead of 2 pi k~ / L)
    import test_oracle_mixed as pm
    orig = bounded.eigenvalues

    def wrong(bc, grid, operator, n, length, h):
        return orig("neumann" if bc == "periodic" else bc, grid, operator, n, length, h)

    monkeypatch.setattr(bounded, "eigenvalues", wrong)
    _fails(pm.test_mixed_ps_closed_form, ["periodic", "dirichlet"], "staggered")


def test_mixed_boundary_node_side_is_caught(monkeypatch):
    # the lower boundary nodes of a REGULAR Dirichlet axis given the upper face
    import test_oracle_mixed as pm
    orig = bounded.mixed_output

    def wrong(psi_inner, bcs, grid, faces):
        out = orig(psi_inner, bcs, grid, faces)
        nd = psi_inner.ndim
        for a in range(nd):
            if bcs[a] == "dirichlet" and grid == "regular" and faces and (a, 1) in faces:
                idx = [slice(None)] * nd
                idx[a] = 0
                out[tuple(idx)] = np.asarray(faces[(a, 1)])
        return out

    monkeypatch.setattr(bounded, "mixed_output", wrong)
    _fails(pm.test_mixed_fd2_matches_dense_solve, ["dirichlet", "neumann", "periodic"], "regular", True)


def test_semi_kernel_sign_is_caught(monkeypatch):
    # the 1D Helmholtz Green's function with the wrong sign
    import test_oracle_semi as ps
    orig = bounded.helmholtz_kernel_1d
    monkeypatch.setattr(bounded, "helmholtz_kernel_1d", lambda kappa, x: -orig(kappa, x))
    _fails(ps.test_semi_fd2_matches_dense_matrix_function, ["unbounded", "periodic"], "staggered")


def test_semi_kernel_decay_is_caught(monkeypatch):
    # exp(-kappa |x| / 2): a decay rate off by a factor of two
    import test_oracle_semi as ps
    orig = bounded.helmholtz_kernel_1d
    monkeypatch.setattr(bounded, "helmholtz_kernel_1d", lambda kappa, x: orig(np.asarray(kappa) / 2.0, x) / 2.0)
    _fails(ps.test_semi_fd2_matches_dense_matrix_function, ["dirichlet", "unbounded"], "regular")


def test_fd_neumann_ghost_sign_is_caught(monkeypatch):
    # the STAGGERED Neumann ghost taken as psi_0 + H g below the lower face
    import test_oracle_fdgrad as pf
    orig = bounded.fd_derivative

    def wrong(psi, bc, grid, h, axis, g_lo=None, g_hi=None):
        if bc == "neumann" and grid == "staggered" and g_lo is not None:
            g_lo = -np.asarray(g_lo)
        return orig(psi, bc, grid, h, axis, g_lo, g_hi)

    monkeypatch.setattr(bounded, "fd_derivative", wrong)
    _fails(pf.test_paraboloid_gradient_is_tfih1dgrad, "neumann", "staggered", 2)


def test_fd_one_sided_coefficient_is_caught(monkeypatch):
    # a first-order one-sided difference on REGULAR Dirichlet boundary nodes
    import test_oracle_fdgrad as pf
    orig = bounded.fd_derivative

    def wrong(psi, bc, grid, h, axis, g_lo=None, g_hi=None):
        out = orig(psi, bc, grid, h, axis, g_lo, g_hi)
        if bc == "dirichlet" and grid == "regular":
            x = np.moveaxis(np.asarray(psi), axis, 0)
            o = np.moveaxis(out, axis, 0)
            o[0] = (x[1] - x[0]) / h
        return out

    monkeypatch.setattr(bounded, "fd_derivative", wrong)
    _fails(pf.test_paraboloid_gradient_is_tfih1dgrad, "dirichlet", "regular", 2)


def test_mixed_periodic_derivative_sign_is_caught(monkeypatch):
    # the periodic axis's first derivative with -i k in place of i k
    import test_oracle_mixed as pm
    orig = bounded.periodic_derivative

    def wrong(psi, length, axis, order=1):
        d = orig(psi, length, axis, order)
        return -d if order == 1 else d

    monkeypatch.setattr(bounded, "periodic_derivative", wrong)
    _fails(pm.test_mixed_gradient_and_laplacian_of_eigenmodes, ["periodic", "dirichlet"], "staggered", "ps")


def test_semi_derivative_kernel_sign_is_caught(monkeypatch):
    # the odd kernel G' of the free-axis derivative with the wrong sign
    import test_oracle_semi as ps
    orig = bounded.helmholtz_kernel_1d_derivative
    monkeypatch.setattr(bounded, "helmholtz_kernel_1d_derivative", lambda kappa, x: -orig(kappa, x))
    _fails(ps.test_semi_gradient_eigenfunction_times_direct_sums, ["unbounded", "periodic"], "staggered")
    _fails(ps.test_semi_free_derivative_second_order, "dirichlet")
