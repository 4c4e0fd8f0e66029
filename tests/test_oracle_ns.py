"""Pins for the compressible Navier-Stokes oracle (CPU only).

The physics (eqs. aRDG_Navier_Stokes, NS_viscosity, NS_heatflux, Sutherland's
law, kappa = Cp mu / Pr) is pinned by textbook flows whose stresses and heat
fluxes are known in closed form:
* simple shear u = (g y, 0): shear stress mu g, no normal stress;
* uniform compression u = (a x, 0): normal stress (4/3) mu a along x and
  -(2/3) mu a across (Stokes' hypothesis), no shear;
* rigid rotation: no stress at all;
* Fourier's law with kappa = Cp mu / Pr for a fluid at rest;
* Sutherland's law: mu(T_ref) = mu_ref, air values at 300/400/500 K against
  standard tables, and the kinetic-theory limit mu ~ T^(1/2) at high T.

The discretisation (weak form, Lax-Friedrichs flux, the aRDG interface viscous
flux on three primitive fields, boundary states) is pinned by:
* a uniform state giving a zero right-hand side;
* a convected density wave (linear fluxes): the right-hand side equals
  -U . grad Q to round-off;
* the moving isentropic vortex (exact Euler solution): the right-hand side
  converges to -U . grad Q;
* steady compressible Couette flow with viscous heating (exact solution of
  the Navier-Stokes equations with constant mu and kappa), in a rotated
  frame: the right-hand side converges to zero;
* the interface reconstruction of u, v and T against the physical-domain
  least-squares brute force;
* conservation: interior faces cancel in the mass-weighted sum;
* planted mistakes in the oracle (CPU) that each of these catches.
"""
import numpy as np
import pytest

import workloads as W
from oracle import ardg
from oracle.ns import Gas, NavierStokes
from oracle.reference_element import mass_1d

from physical_bruteforce import ParallelogramLS, PhysPoly


# ----------------------------------------------------------------------------
# exact solutions
# ----------------------------------------------------------------------------

def couette(gas, U=0.5, h=10.0, T0=1.0, p0=1.0, theta=0.5, x0=(0.0, -5.0)):
    """Steady plane Couette flow with viscous heating, walls at eta = 0 and h
    moving at 0 and U, both at T0, rotated by theta.  Momentum: mu u'' = 0;
    energy: kappa T'' + mu u'^2 = 0, so T = T0 + Pr U^2/(2 Cp) (eta/h)(1 - eta/h);
    p constant, rho = p / (R T)."""
    c, s = np.cos(theta), np.sin(theta)

    def Q(x, y, t=0.0):
        eta = -s * (x - x0[0]) + c * (y - x0[1])
        un = U * eta / h
        T = T0 + gas.Pr * U * U / (2 * gas.cp) * (eta / h) * (1 - eta / h)
        rho = p0 / (gas.R * T)
        u, v = un * c, un * s
        E = p0 / (gas.gamma - 1) + 0.5 * rho * (u * u + v * v)
        return np.stack([rho, rho * u, rho * v, E])
    return Q


def vortex(gas, beta=5.0, uinf=(0.5, 0.3), c0=(5.0, 0.0), L=2.5):
    """The isentropic vortex convected at uinf (exact Euler solution, R = 1)."""
    g = gas.gamma

    def Q(x, y, t=0.0):
        xc, yc = (x - c0[0] - uinf[0] * t) / L, (y - c0[1] - uinf[1] * t) / L
        f = np.exp(0.5 * (1 - xc * xc - yc * yc))
        u = uinf[0] - beta / (2 * np.pi) * f * yc
        v = uinf[1] + beta / (2 * np.pi) * f * xc
        T = 1 - (g - 1) * beta ** 2 / (8 * g * np.pi ** 2) * f * f
        rho = T ** (1 / (g - 1))
        p = rho * T
        return np.stack([rho, rho * u, rho * v, p / (g - 1) + 0.5 * rho * (u * u + v * v)])

    def dQdt(x, y, h=1e-30):
        # complex-step derivative in t (exact to round-off)
        return np.imag(Q(x + 0j, y + 0j, 1j * h)) / h
    return Q, dQdt


def density_wave(gas, U=(0.4, -0.25), p0=1.0, a=(0.05, 0.03), rho0=1.0):
    """rho linear in x and y, velocity and pressure constant: every flux is
    linear, and dQ/dt = -U . grad Q exactly."""
    def Q(x, y, t=0.0):
        rho = rho0 + a[0] * (x - U[0] * t) + a[1] * (y - U[1] * t)
        E = p0 / (gas.gamma - 1) + 0.5 * rho * (U[0] ** 2 + U[1] ** 2)
        return np.stack([rho, rho * U[0], rho * U[1], E])

    def dQdt(x, y, h=1e-30):
        return np.imag(Q(x + 0j, y + 0j, 1j * h)) / h
    return Q, dQdt


def _system(kind, n, N, gas, Qf):
    m = W.paper_grid(kind, n)
    ns = NavierStokes(m.vxy, m.etov, N, gas, Qf)
    xy = ns.nodal_xy()
    return ns, xy, Qf(xy[..., 0], xy[..., 1])


# ----------------------------------------------------------------------------
# physics pins
# ----------------------------------------------------------------------------

def _stress(gas, ux, uy, vx, vy, mu_T=1.0):
    z = np.zeros(1)
    one = np.ones(1)
    Gx, Gy = gas.viscous(0 * one, 0 * one, mu_T * one, ux + z, uy + z, vx + z, vy + z, z, z)
    # momentum rows of G are -Pi
    return -Gx[1, 0], -Gx[2, 0], -Gy[1, 0], -Gy[2, 0]


def test_simple_shear_stress():
    gas = Gas(mu_ref=0.3, law="constant")
    Pxx, Pxy, Pyx, Pyy = _stress(gas, 0.0, 2.0, 0.0, 0.0)
    assert Pxy == pytest.approx(0.6) and Pyx == pytest.approx(0.6)
    assert Pxx == pytest.approx(0.0, abs=1e-15) and Pyy == pytest.approx(0.0, abs=1e-15)


def test_uniform_compression_stresses():
    gas = Gas(mu_ref=0.3, law="constant")
    Pxx, Pxy, _, Pyy = _stress(gas, -1.5, 0.0, 0.0, 0.0)
    assert Pxx == pytest.approx(4.0 / 3.0 * 0.3 * -1.5)
    assert Pyy == pytest.approx(-2.0 / 3.0 * 0.3 * -1.5)
    assert Pxy == pytest.approx(0.0, abs=1e-15)


def test_rigid_rotation_is_stress_free():
    gas = Gas(mu_ref=0.3, law="constant")
    assert np.allclose(_stress(gas, 0.0, -0.7, 0.7, 0.0), 0.0, atol=1e-15)


def test_fourier_heat_flux_and_viscous_work():
    gas = Gas(mu_ref=0.2, law="constant", Pr=0.7)
    z, one = np.zeros(1), np.ones(1)
    # fluid at rest, T gradient (3, -2): energy flux q = -Cp mu / Pr grad T
    Gx, Gy = gas.viscous(z, z, one, z, z, z, z, 3 * one, -2 * one)
    kappa = gas.gamma * gas.R / (gas.gamma - 1) * 0.2 / 0.7
    assert Gx[3, 0] == pytest.approx(-3 * kappa) and Gy[3, 0] == pytest.approx(2 * kappa)
    assert np.allclose(Gx[:3], 0) and np.allclose(Gy[:3], 0)
    # shear flow at speed 1.5 along x with du/dy = 2: the viscous work
    # u tau_xy = 1.5 * 0.2 * 2 leaves through the y faces (energy flux -u tau)
    Gx, Gy = gas.viscous(1.5 * one, z, one, z, 2 * one, z, z, z, z)
    assert Gy[3, 0] == pytest.approx(-1.5 * 0.2 * 2)


def test_sutherland_air():
    air = Gas(mu_ref=1.716e-5, T_ref=273.15, S=110.4, R=287.0)
    assert air.mu(273.15) == pytest.approx(1.716e-5, rel=1e-14)
    # tabulated dynamic viscosity of air at 1 atm (Pa s)
    for T, table in ((300.0, 1.846e-5), (400.0, 2.301e-5), (500.0, 2.701e-5)):
        assert air.mu(T) == pytest.approx(table, rel=0.015)
    # high-temperature limit: mu grows like T^(1/2)
    assert air.mu(4e8) / air.mu(1e8) == pytest.approx(2.0, rel=1e-5)


# ----------------------------------------------------------------------------
# discretisation pins
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("kind", ["a", "c"])
def test_uniform_state_has_zero_rhs(kind):
    gas = Gas()
    Q0 = np.array([1.2, 0.3, -0.2, 2.5])
    ns, xy, _ = _system(kind, 2, 3, gas,
                        lambda x, y, t=0.0: Q0.reshape((4,) + (1,) * np.ndim(x)) + 0 * x)
    Q = np.broadcast_to(Q0[:, None, None], (4, ns.geom.K, ns.ops.Np)).copy()
    assert np.abs(ns.rhs(Q)).max() < 1e-13


@pytest.mark.parametrize("N", [1, 2, 3])
def test_density_wave_is_exact(N):
    # inviscid: T = p / (rho R) varies with rho, so heat conduction would act
    gas = Gas(mu_ref=0.0, law="constant")
    Qf, dQ = density_wave(gas)
    ns, xy, Q = _system("c", 2, N, gas, Qf)
    ex = dQ(xy[..., 0], xy[..., 1])
    assert np.abs(ns.rhs(Q) - ex).max() < 1e-13


def _vortex_errors(N, levels, gas=None, ns_cls=NavierStokes):
    gas = gas or Gas(mu_ref=0.0, law="constant")
    Qf, dQ = vortex(gas)
    out = []
    for n in levels:
        m = W.paper_grid("b", n)
        ns = ns_cls(m.vxy, m.etov, N, gas, Qf)
        xy = ns.nodal_xy()
        Q = Qf(xy[..., 0], xy[..., 1])
        out.append(np.abs(ns.rhs(Q) - dQ(xy[..., 0], xy[..., 1])).max())
    return np.array(out)


def test_vortex_rhs_converges():
    e = _vortex_errors(3, [2, 4, 8])
    assert np.all(e[:-1] / e[1:] > 3.5), e
    assert e[-1] < 0.03


def _couette_residuals(N, levels, gas=None, ns_cls=NavierStokes, theta=0.5):
    gas = gas or Gas(mu_ref=0.05, law="constant")
    Qf = couette(gas, theta=theta)
    out = []
    for n in levels:
        m = W.paper_grid("a", n)
        ns = ns_cls(m.vxy, m.etov, N, gas, lambda x, y, t: Qf(x, y))
        xy = ns.nodal_xy()
        out.append(np.abs(ns.rhs(Qf(xy[..., 0], xy[..., 1]))).max(axis=(1, 2)))
    return np.array(out)


@pytest.mark.parametrize("N,rate", [(2, 1.6), (3, 2.6)])
def test_couette_steady_residual_converges(N, rate):
    e = _couette_residuals(N, [2, 4, 8])
    rates = np.log2(e[:-1] / e[1:])
    assert np.all(rates > rate), rates
    assert e[-1].max() < (3e-5 if N == 2 else 2e-7)


def test_interface_reconstruction_matches_physical_bruteforce():
    """u~, v~ and T~ at the diagonal nodes and their gradients, interior and
    boundary edges of a distorted grid, against the least-squares fit built
    in physical coordinates."""
    N = 3
    gas = Gas()
    Qf, _ = vortex(gas, L=1.5)
    ns, xy, Q = _system("c", 1, N, gas, Qf)
    rng = np.random.default_rng(7)
    Q = Q * (1 + 0.05 * rng.standard_normal(Q.shape))
    _, u, v, _, T = gas.primitives(Q)
    g = ns.geom
    checked = 0
    n_int, n_bdy = min(6, len(g.interior)), min(4, len(g.boundary))
    for e, (k1, f1, k2, f2) in enumerate(g.interior[:n_int]):
        eg = ns.int_geom[e]
        T1 = ardg.total_projection(ns.ops, eg.pi1, f1)
        T2 = ardg.total_projection(ns.ops, eg.pi2, f2)
        ls = ParallelogramLS(N, eg)
        D = ls.diagonal()
        for p in (u, v, T):
            val, gx, gy = ns._recon(eg, T1 @ p[k1], T2 @ p[k2])
            c = ls.fit(PhysPoly(N, xy[k1], p[k1]), PhysPoly(N, xy[k2], p[k2]))
            assert np.allclose(val, ls.value(c, D), atol=1e-11)
            G = ls.grad(c, D)
            assert np.allclose(gx, G[:, 0], atol=1e-10) and np.allclose(gy, G[:, 1], atol=1e-10)
            checked += 1
    for e, (k1, f1) in enumerate(g.boundary[:n_bdy]):
        eg = ns.bdy_geom[e]
        T1 = ardg.total_projection(ns.ops, eg.pi1, f1)
        ls = ParallelogramLS(N, eg)
        X2 = ardg.ghost_nodes(N, eg)
        _, ug, vg, _, Tg = gas.primitives(Qf(X2[:, 0], X2[:, 1]))
        D = ls.diagonal()
        for p, pg in zip((u, v, T), (ug, vg, Tg)):
            val, gx, gy = ns._recon(eg, T1 @ p[k1], ns.ops.Vinv @ pg)
            c = ls.fit(PhysPoly(N, xy[k1], p[k1]), PhysPoly(N, X2, pg))
            assert np.allclose(val, ls.value(c, D), atol=1e-11)
            G = ls.grad(c, D)
            assert np.allclose(gx, G[:, 0], atol=1e-10) and np.allclose(gy, G[:, 1], atol=1e-10)
            checked += 1
    assert checked == 3 * (n_int + n_bdy) >= 18


def test_interior_faces_cancel():
    """sum_k int_k dQ/dt = -(boundary flux integral): with M the mass matrix
    and w the 1D Gauss-Lobatto weights on faces."""
    N = 3
    gas = Gas()
    Qf, _ = vortex(gas, L=1.5)
    ns, xy, Q = _system("c", 2, N, gas, Qf)
    rng = np.random.default_rng(3)
    Q = Q * (1 + 0.05 * rng.standard_normal(Q.shape))
    r = ns.rhs(Q)
    ops, g = ns.ops, ns.geom
    total = np.einsum("k,ckn->c", g.J, r @ ops.M.T)     # sum_k 1^T M J dQ/dt
    # boundary integral of H* . n: the face quadrature is the 1D mass matrix
    Hs = ns.face_fluxes(Q, 0.0)
    wf = mass_1d(N) @ np.ones(ops.Nfp)
    bnd = np.zeros(4)
    for (k, f) in g.boundary:
        bnd += g.sJ[k, f] * (Hs[k, f] @ wf)
    assert np.allclose(total, -bnd, atol=1e-11 * np.abs(bnd).max()), (total, -bnd)


# ----------------------------------------------------------------------------
# planted mistakes (in the oracle, on the CPU)
# ----------------------------------------------------------------------------

class _WorkSignFlipped(Gas):
    def viscous(self, *a):
        Gx, Gy = super().viscous(*a)
        u, v, T, ux, uy, vx, vy, Tx, Ty = a
        mu = self.mu(T)
        div = ux + vy
        Pxx, Pyy, Pxy = mu * (2 * ux - 2 / 3 * div), mu * (2 * vy - 2 / 3 * div), mu * (uy + vx)
        Gx[3] += 2 * (u * Pxx + v * Pxy)
        Gy[3] += 2 * (u * Pxy + v * Pyy)
        return Gx, Gy


class _NoPressureInXMomentum(Gas):
    def inviscid(self, Q):
        Fx, Fy = super().inviscid(Q)
        Fx[1] -= self.primitives(Q)[3]
        return Fx, Fy


class _TemperatureFromU(NavierStokes):
    def _primitive_fields(self, Q):
        u, v, T = super()._primitive_fields(Q)
        return [u, v, u]


def test_planted_viscous_work_sign_is_caught():
    gas = _WorkSignFlipped(mu_ref=0.05, law="constant")
    e = _couette_residuals(3, [2, 4], gas=gas)
    assert e[-1, 3] > 1e-4 and e[0, 3] / e[1, 3] < 2.5


def test_planted_missing_pressure_is_caught():
    e = _vortex_errors(3, [2, 4], gas=_NoPressureInXMomentum(mu_ref=0.0, law="constant"))
    assert e[-1] > 0.1


def test_planted_wrong_interface_field_is_caught():
    e = _couette_residuals(3, [2, 4], ns_cls=_TemperatureFromU)
    assert e[-1].max() > 1e-4
