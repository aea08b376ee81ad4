"""FP64 CPU oracle of one time step of the thermal pseudopotential D3Q19 scheme.

TEST INFRASTRUCTURE ONLY.  Nothing on the product path may import this
module: only the test suite, the smoke check and the CPU baseline leg of the
benchmark use it.  It shares no code, table or helper with the HIP library.

What it computes follows Biferale, Perlekar, Sbragaglia & Toschi,
"Convection in multiphase flows using Lattice Boltzmann methods"
(arXiv:1111.0905), section "Algorithm":

* eq. (LBEQ)/(LBEQ2): two BGK lattice Boltzmann equations, f for mass and
  momentum (relaxation time tau_nu), g for rho*T (relaxation time tau_kappa);
* eq. (HYDRO): rho = sum f, rho u = sum c f, rho T = sum g;
* velocity shift u' = u + tau_nu F / rho inside f^eq;
* eq. (FORCE): F = -G sum_l W(|c_l|^2) c_l psi(x) psi(x + c_l) with
  psi = exp(-1/rho) and weights isotropic to 4th order;
* the f/g coupling: the second moment of f^eq is rho T delta + rho u u;
* a counter-term in the g dynamics restoring P0 div(u) of the second form of
  the temperature equation (eq. (eq));
* gravity g rho z-hat in the momentum equation (eq. (ns)), no-slip walls at
  the bottom and top, periodic horizontal directions (Fig. 1 caption), and
  imposed wall temperatures T_d (bottom) and T_u (top).

The paper prints neither the equilibria, nor the counter-term, nor the wall
rules.  The readings used here (each stated where it is used) are:

* force weights W = 1/6 (axis) and 1/12 (face diagonal), i.e. sum W c c = 1;
  then the bulk non-ideal pressure is (G/2) exp(-2/rho), rho_c = 1,
  T_c = -G / e^2;
* f^eq(u', rho) is the second-order polynomial equilibrium whose isotropic
  second moment is rho T_lat (a constant lattice temperature, by default the
  mean wall temperature, set through the rest population); the dynamical
  temperature enters the f dynamics through the force
  F_T = -grad(rho T - rho T_lat), so that for G -> 0 the momentum equation
  sees the second moment rho T delta + rho u u (the f/g coupling);
* g^eq(u, F, T): polynomial equilibrium of E = rho T whose first moment is
  gamma E v (gamma = 1 + 1/c_v; v = (j + F/2)/rho carries the force) and
  whose second moment has the isotropic part c_s^2 rho_kappa T, giving one
  conductivity kappa = c_v c_s^2 (tau_kappa - 1/2) rho_kappa in both phases
  (Table 1);
* counter-term: the factor gamma in the flux plus the source
  S = (1/c_v) v . grad E added as w_l S after the g collision; together
  they give dE/dt + div(E v) = -(E/c_v) div v + (kappa/c_v) lap T, i.e.
  the second form of eq. (eq);
* v = (j + F/2)/rho is the physical velocity;
* gravity as a body force rho (0, 0, -g) added to F;
* half-way bounce-back for f and anti-bounce-back for g at the walls, which
  sit half a lattice spacing below k = 0 and above k = nz - 1;
* ghost planes at the walls for the gradient stencils: psi from the mirror
  image of rho (neutral wetting), or, where a wall density is given (the
  paper is silent on wettability), psi of that density; E and rho in the
  thermal force and in S
  extrapolated linearly through the wall (a conductive state at rest is then
  an exact steady state with Nu = 1).

A literal reading that puts the dynamical T into the rest population of
f^eq and adds the counter-term as -(E/c_v) div v is linearly unstable at the
paper's viscosity; the readings above are linearly stable there for critical
temperatures T_c <~ 0.05 (the default; see the stability test).  With the
constant T_lat in f^eq only the small part rho (T - T_lat) of the ideal
pressure goes through the stencil force, which keeps the coexistence
densities on the Maxwell construction (Fig. 1).

Populations are stored as tensors of shape (19, nz, ny, nx), fields as
(nz, ny, nx), vectors as (3, nz, ny, nx); all float64 on the CPU.  Every
function is written with torch operations so that autograd of step() is the
discrete adjoint of the scheme.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, replace

import torch

DT = torch.float64

# D3Q19 velocity set: rest, 6 axis, 12 face diagonals; opposite pairs are
# (1,2), (3,4), ..., (17,18).
_C_LIST = [
    (0, 0, 0),
    (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1),
    (1, 1, 0), (-1, -1, 0), (1, -1, 0), (-1, 1, 0),
    (1, 0, 1), (-1, 0, -1), (1, 0, -1), (-1, 0, 1),
    (0, 1, 1), (0, -1, -1), (0, 1, -1), (0, -1, 1),
]
Q19 = 19
C_INT = _C_LIST
C = torch.tensor(_C_LIST, dtype=DT)                       # (19, 3)
OPP = [0] + [l + 1 if l % 2 == 1 else l - 1 for l in range(1, 19)]
# lattice weights (textbook D3Q19), c_s^2 = 1/3
W_LAT = torch.tensor([1.0 / 3.0] + [1.0 / 18.0] * 6 + [1.0 / 36.0] * 12, dtype=DT)
# pseudopotential-force weights, isotropic to 4th order, sum W c c = identity
W_FOR = torch.tensor([0.0] + [1.0 / 6.0] * 6 + [1.0 / 12.0] * 12, dtype=DT)
# isotropic second-moment adjusters of f^eq (a) and g^eq (b)
A_F = torch.tensor([-2.0] + [3.0 / 18.0] * 6 + [3.0 / 36.0] * 12, dtype=DT)
B_G = torch.tensor([-2.0 / 3.0] + [1.0 / 18.0] * 6 + [1.0 / 36.0] * 12, dtype=DT)
CS2 = 1.0 / 3.0


@dataclass(frozen=True)
class Params:
    """Problem statement of the convection cell (eqs. (ns), (LBEQ)-(FORCE))."""
    nx: int
    ny: int
    nz: int
    tau_nu: float = 1.0
    tau_kappa: float = 1.0
    G: float = -0.05 * math.e ** 2
    T_d: float = 0.0475
    T_u: float = 0.0425
    gravity: float = 0.0
    c_v: float = 1.0
    rho_kappa: float = 0.5
    periodic_z: bool = False
    T_lat: float = 0.0          # lattice temperature of f^eq; 0 -> (T_d + T_u) / 2
    # wetting (the paper is silent on wettability): a wall density > 0 gives
    # the psi ghost plane beyond that wall the constant psi(rho_wall), the
    # wall-density method of Benzi et al., Phys. Rev. E 74, 021509 (2006);
    # <= 0 mirrors psi of the wall plane (neutral wetting)
    rho_wall_d: float = 0.0
    rho_wall_u: float = 0.0
    # form of the pseudopotential: 0 = exp(-1/rho), the paper's choice; 1 =
    # 1 - exp(-rho), the original Shan-Chen form, one of the alternatives the
    # paper names as prior art (its coexistence follows the mechanical rule of
    # that psi, not Maxwell's)
    psi_form: int = 0

    def with_(self, **kw) -> "Params":
        return replace(self, **kw)

    @property
    def kappa(self) -> float:
        """Thermal conductivity realised by the g equilibrium."""
        return self.c_v * CS2 * (self.tau_kappa - 0.5) * self.rho_kappa

    @property
    def nu(self) -> float:
        """Kinematic viscosity of the f equation."""
        return CS2 * (self.tau_nu - 0.5)

    @property
    def T_c(self) -> float:
        return -self.G / math.e ** 2

    @property
    def T_lattice(self) -> float:
        return self.T_lat if self.T_lat > 0 else 0.5 * (self.T_d + self.T_u)


# ---------------------------------------------------------------- stencils

def _pad_z(a: torch.Tensor, walls: bool, odd: bool) -> torch.Tensor:
    """One ghost plane below k=0 and above k=nz-1 (dim -3).

    Walls: mirror through the half-way wall (sign flip if odd).
    Periodic: wrap around.
    """
    if walls:
        lo, hi = a[..., :1, :, :], a[..., -1:, :, :]
        if odd:
            lo, hi = -lo, -hi
    else:
        lo, hi = a[..., -1:, :, :], a[..., :1, :, :]
    return torch.cat([lo, a, hi], dim=-3)


def _at(a_pad: torch.Tensor, c) -> torch.Tensor:
    """Value at x + c for every node x, from a z-padded field."""
    cx, cy, cz = c
    nz = a_pad.shape[-3] - 2
    s = a_pad[..., 1 + cz:1 + cz + nz, :, :]
    return torch.roll(s, shifts=(-cy, -cx), dims=(-2, -1))


# ---------------------------------------------------------------- moments

def hydro_moments(f: torch.Tensor, g: torch.Tensor):
    """eq. (HYDRO): rho = sum f, j = sum c f, E = rho T = sum g."""
    rho = f.sum(0)
    j = torch.einsum("la,lzyx->azyx", C, f)
    E = g.sum(0)
    return rho, j, E


def pseudopotential(rho: torch.Tensor, form: int = 0) -> torch.Tensor:
    """psi[rho] = exp(-1/rho), the choice the paper makes for thermodynamic
    consistency (form 0), or the original Shan-Chen 1 - exp(-rho) (form 1)."""
    if form == 1:
        return 1.0 - torch.exp(-rho)
    return torch.exp(-1.0 / rho)


def _psi_scalar(rho: float, form: int) -> float:
    return 1.0 - math.exp(-rho) if form == 1 else math.exp(-1.0 / rho)


def _pad_z_linear(a: torch.Tensor, walls: bool) -> torch.Tensor:
    """Ghost planes extrapolated linearly through the walls,
    a(-1) = 2 a(0) - a(1) (needs nz >= 2); periodic wrap without walls."""
    if not walls:
        return _pad_z(a, walls=False, odd=False)
    lo = 2.0 * a[..., :1, :, :] - a[..., 1:2, :, :]
    hi = 2.0 * a[..., -1:, :, :] - a[..., -2:-1, :, :]
    return torch.cat([lo, a, hi], dim=-3)


def _grad_w(p: Params, a: torch.Tensor, ghost: str = "mirror") -> torch.Tensor:
    """sum_l W_l c_l a(x + c_l): the W-stencil central gradient (2nd order,
    isotropic to 4th order).  At the walls the ghost plane is the mirror
    image ("mirror") or the linear extrapolation ("linear") of the field."""
    if ghost == "mirror":
        ap = _pad_z(a, walls=not p.periodic_z, odd=False)
    else:
        ap = _pad_z_linear(a, walls=not p.periodic_z)
    s = torch.zeros((3,) + tuple(a.shape), dtype=a.dtype)
    for l in range(1, Q19):
        s = s + W_FOR[l] * C[l].view(3, 1, 1, 1) * _at(ap, C_INT[l])
    return s


def _grad_w_psi(p: Params, psi: torch.Tensor) -> torch.Tensor:
    """W-stencil gradient of psi; at a wall with a prescribed density the
    ghost plane holds psi(rho_wall), elsewhere the mirror image."""
    if p.periodic_z or (p.rho_wall_d <= 0 and p.rho_wall_u <= 0):
        return _grad_w(p, psi)
    ap = _pad_z(psi, walls=True, odd=False)
    lo, mid, hi = ap[..., :1, :, :], ap[..., 1:-1, :, :], ap[..., -1:, :, :]
    if p.rho_wall_d > 0:
        lo = torch.full_like(lo, _psi_scalar(p.rho_wall_d, p.psi_form))
    if p.rho_wall_u > 0:
        hi = torch.full_like(hi, _psi_scalar(p.rho_wall_u, p.psi_form))
    ap = torch.cat([lo, mid, hi], dim=-3)
    s = torch.zeros((3,) + tuple(psi.shape), dtype=psi.dtype)
    for l in range(1, Q19):
        s = s + W_FOR[l] * C[l].view(3, 1, 1, 1) * _at(ap, C_INT[l])
    return s


def sc_force(p: Params, rho: torch.Tensor, G=None) -> torch.Tensor:
    """eq. (FORCE): F_SC = -G psi(x) sum_l W_l c_l psi(x + c_l)."""
    G = p.G if G is None else G
    psi = pseudopotential(rho, p.psi_form)
    return -G * psi * _grad_w_psi(p, psi)


def forces(p: Params, rho, E, G=None):
    """Total force on the f populations and the two gradients the g update
    needs.

    F = F_SC + F_T + rho (0, 0, -g), where F_T = -grad[rho T - rho T_lat]
    adds to the lattice pressure rho T_lat of f^eq the rest of the ideal
    pressure rho T (T taken from the g populations): in the limit G -> 0 the
    f dynamics then carries the second moment rho T delta + rho u u.  The
    gradients of E and rho use ghost planes extrapolated linearly through the
    walls (psi uses the mirror image).
    """
    gE = _grad_w(p, E, "linear")
    grho = _grad_w(p, rho, "linear")
    F = sc_force(p, rho, G) - (gE - p.T_lattice * grho)
    F = F + torch.stack([torch.zeros_like(rho), torch.zeros_like(rho), -p.gravity * rho])
    return F, gE, grho


def f_equilibrium(rho, u, T_lat=CS2) -> torch.Tensor:
    """f^eq_l(u', rho): second-order polynomial equilibrium of the D3Q19
    lattice with moments rho, rho u, rho T_lat delta + rho u u (the rest
    population carries rho (T_lat - c_s^2) a_l, a_0 = -2, a_l = 3 w_l)."""
    cu = torch.einsum("la,azyx->lzyx", C, u)
    uu = (u * u).sum(0)
    w = W_LAT.view(Q19, 1, 1, 1)
    a = A_F.view(Q19, 1, 1, 1)
    return w * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu) + a * rho * (T_lat - CS2)


def g_equilibrium(p: Params, rho, E, v, T, v_lin=None) -> torch.Tensor:
    """g^eq_l(u, F, T) with moments
      sum g^eq = E = rho T,
      sum c g^eq = gamma E v,   gamma = 1 + 1/c_v,
      sum c c g^eq = c_s^2 rho_kappa T delta + gamma E v v,
    where v = (j + F/2)/rho carries the force.  The isotropic part of the
    second moment sets one conductivity kappa = c_v c_s^2 (tau_kappa - 1/2)
    rho_kappa in both phases; the factor gamma carries the compressive work
    P0 div u (counter-term, flux part).  v_lin, if given, replaces v in the
    linear term only (used by the moment tests)."""
    v_lin = v if v_lin is None else v_lin
    gam = 1.0 + 1.0 / p.c_v
    cl = torch.einsum("la,azyx->lzyx", C, v_lin)
    cv = torch.einsum("la,azyx->lzyx", C, v)
    vv = (v * v).sum(0)
    w = W_LAT.view(Q19, 1, 1, 1)
    b = B_G.view(Q19, 1, 1, 1)
    return w * (E + gam * E * (3.0 * cl + 4.5 * cv * cv - 1.5 * vv)) + b * (p.rho_kappa - rho) * T


def macroscopic(p: Params, f: torch.Tensor, g: torch.Tensor, G=None) -> dict:
    """All node-local quantities of one step, at the current time level.

    u_shift = u + tau_nu F / rho (velocity shift, Algorithm section);
    v = (j + F/2) / rho, the physical velocity;
    S = (1/c_v) v . grad E, the source part of the counter-term: with the
      flux gamma E v of g^eq it gives
      dE/dt + div(E v) = -(E/c_v) div v + (kappa/c_v) lap T.
    """
    rho, j, E = hydro_moments(f, g)
    T = E / rho
    F, gE, _ = forces(p, rho, E, G)
    u_shift = (j + p.tau_nu * F) / rho
    v = (j + 0.5 * F) / rho
    S = (v * gE).sum(0) / p.c_v
    return dict(rho=rho, j=j, E=E, T=T, F=F, u_shift=u_shift, v=v, S=S, gradE=gE)


# ---------------------------------------------------------------- the step

def collide(p: Params, f, g, G=None):
    """Right-hand sides of eqs. (LBEQ)/(LBEQ2) plus the counter-term source."""
    m = macroscopic(p, f, g, G)
    feq = f_equilibrium(m["rho"], m["u_shift"], p.T_lattice)
    geq = g_equilibrium(p, m["rho"], m["E"], m["v"], m["T"])
    fs = f - (f - feq) / p.tau_nu
    gs = g - (g - geq) / p.tau_kappa + W_LAT.view(Q19, 1, 1, 1) * m["S"]
    return fs, gs


def stream(p: Params, fs, gs, T_d=None, T_u=None):
    """Left-hand sides of eqs. (LBEQ)/(LBEQ2): f_l(x + c_l, t+1) = f*_l(x).

    Periodic in x, y.  With walls, a population whose destination leaves
    0 <= k < nz returns to its own node in the opposite direction (half-way
    bounce-back for f; anti-bounce-back about w_l rho_kappa T_wall for g).
    """
    T_d = p.T_d if T_d is None else T_d
    T_u = p.T_u if T_u is None else T_u
    nf, ng = [], []
    for l in range(Q19):
        cx, cy, cz = C_INT[l]
        a = torch.roll(fs[l], shifts=(cy, cx), dims=(1, 2))
        b = torch.roll(gs[l], shifts=(cy, cx), dims=(1, 2))
        if cz == 0:
            pass
        elif p.periodic_z:
            a = torch.roll(a, shifts=cz, dims=0)
            b = torch.roll(b, shifts=cz, dims=0)
        else:
            o = OPP[l]
            wr = 2.0 * W_LAT[l] * p.rho_kappa
            if cz == 1:   # enters from below: source plane -1 is the bottom wall
                a = torch.cat([fs[o][:1], a[:-1]], dim=0)
                b = torch.cat([-gs[o][:1] + wr * T_d, b[:-1]], dim=0)
            else:         # enters from above: source plane nz is the top wall
                a = torch.cat([a[1:], fs[o][-1:]], dim=0)
                b = torch.cat([b[1:], -gs[o][-1:] + wr * T_u], dim=0)
        nf.append(a)
        ng.append(b)
    return torch.stack(nf), torch.stack(ng)


def step(p: Params, f, g, G=None, T_d=None):
    """One time step t -> t+1 of the post-streaming state (f, g)."""
    fs, gs = collide(p, f, g, G)
    return stream(p, fs, gs, T_d=T_d)


# ---------------------------------------------------------------- init

def initial_temperature(p: Params, T_d=None) -> torch.Tensor:
    """Linear conduction profile between the half-way walls:
    T0(k) = T_d + (T_u - T_d) (k + 1/2) / nz."""
    T_d = p.T_d if T_d is None else T_d
    k = torch.arange(p.nz, dtype=DT)
    Tz = T_d + (p.T_u - T_d) * (k + 0.5) / p.nz
    return Tz.view(p.nz, 1, 1).expand(p.nz, p.ny, p.nx)


def init_state(p: Params, rho0, T0=None):
    """Local equilibrium at rest: f = f^eq(rho0, 0), g = g^eq(rho0 T0, v = 0)."""
    rho0 = torch.as_tensor(rho0, dtype=DT)
    T0 = initial_temperature(p) if T0 is None else torch.as_tensor(T0, dtype=DT)
    zero = torch.zeros((3,) + tuple(rho0.shape), dtype=DT)
    f = f_equilibrium(rho0, zero, p.T_lattice)
    g = g_equilibrium(p, rho0, rho0 * T0, zero, T0)
    return f, g


# ---------------------------------------------------------------- diagnostics

def internal_energy(p: Params, rho, T):
    """U = c_v T + integral of P_NI / rho^2 d rho = c_v T + (G/4) exp(-2/rho),
    for the bulk non-ideal pressure P_NI = (G/2) exp(-2/rho)."""
    return p.c_v * T + 0.25 * p.G * torch.exp(-2.0 / rho)


def totals(p: Params, f, g) -> torch.Tensor:
    """[M, Px, Py, Pz, sum rho T, sum rho U]; momentum is sum rho v."""
    m = macroscopic(p, f, g)
    rU = m["rho"] * internal_energy(p, m["rho"], m["T"])
    P = (m["rho"] * m["v"]).sum(dim=(1, 2, 3))
    return torch.stack([m["rho"].sum(), P[0], P[1], P[2], m["E"].sum(), rU.sum()])


def bulk_pressure(p: Params, rho, T):
    """Equation of state (text after eq. (ns)): P = P0 + P_NI with P0 = rho T
    and P_NI = (G/2) psi^2, i.e. (G/2) exp(-2/rho) for the paper's psi (its
    G exp(-2/rho) with the factor 1/2 of the W-normalised force)."""
    psi = pseudopotential(rho, p.psi_form)
    return rho * T + 0.5 * p.G * psi * psi


def divergence(p: Params, v: torch.Tensor) -> torch.Tensor:
    """sum_l W_l c_l . v(x + c_l): the W-stencil divergence (central, like
    the gradients).  At the no-slip walls the ghost planes hold the negative
    mirror image of every velocity component (v = 0 on the half-way wall)."""
    vp = _pad_z(v, walls=not p.periodic_z, odd=True)
    s = torch.zeros(tuple(v.shape[1:]), dtype=v.dtype)
    for l in range(1, Q19):
        cv = sum(C_INT[l][a] * _at(vp[a], C_INT[l]) for a in range(3) if C_INT[l][a])
        s = s + W_FOR[l] * cv
    return s


def pressure_work(p: Params, f, g):
    """Horizontal average of P d_j u_j at each k: the source of the layer
    heat balance eq. (heat2) and the integrand of the constraint eq. (flux),
    Nu(z) - Nu(0) = -integral_0^z <P d_j u_j>.  u is the physical velocity
    v = (j + F/2)/rho, P the bulk equation of state."""
    m = macroscopic(p, f, g)
    P = bulk_pressure(p, m["rho"], m["T"])
    return (P * divergence(p, m["v"])).mean(dim=(1, 2))


def plane_profiles(p: Params, f, g):
    """Horizontal averages at each k: T-bar(k) and <rho U v_z>(k)."""
    m = macroscopic(p, f, g)
    rUv = m["rho"] * internal_energy(p, m["rho"], m["T"]) * m["v"][2]
    return m["T"].mean(dim=(1, 2)), rUv.mean(dim=(1, 2))


def nusselt(p: Params, f, g):
    """Wall and z-dependent Nusselt numbers (eq. (flux), Fig. 2 bottom).

    Wall flux from the half-cell one-sided difference between the wall
    temperature and the first plane; Nu(k) = [<rho U v_z> - kappa dT/dz](k)
    in units of kappa (T_d - T_u) / nz, with a central difference and ghost
    planes linear through the walls.
    """
    Tz, rUv = plane_profiles(p, f, g)
    dT = p.T_d - p.T_u
    nz = p.nz
    nu_bot = 2.0 * nz * (p.T_d - Tz[0]) / dT
    nu_top = 2.0 * nz * (Tz[-1] - p.T_u) / dT
    Tg = torch.cat([(2.0 * p.T_d - Tz[0]).view(1), Tz, (2.0 * p.T_u - Tz[-1]).view(1)])
    dTdz = 0.5 * (Tg[2:] - Tg[:-2])
    nu_z = (rUv - p.kappa * dTdz) * nz / (p.kappa * dT)
    return nu_bot, nu_top, nu_z, Tz


def q_bottom(p: Params, f, g, T_d=None):
    """Plane-averaged conductive heat flux through the bottom wall,
    2 kappa (T_d - T-bar(0))."""
    T_d = p.T_d if T_d is None else T_d
    rho, _, E = hydro_moments(f[:, :1], g[:, :1])
    return 2.0 * p.kappa * (T_d - (E / rho).mean())


# ---------------------------------------------------------------- driver

class Oracle:
    """Stateful wrapper mirroring the C interface: init / step(n) /
    moments / nusselt / get_state / set_state."""

    def __init__(self, p: Params, rho0=None, f=None, g=None):
        self.p = p
        if f is not None:
            self.f = torch.as_tensor(f, dtype=DT).clone()
            self.g = torch.as_tensor(g, dtype=DT).clone()
        else:
            self.f, self.g = init_state(p, rho0)
        self.t = 0

    def step(self, n: int = 1):
        with torch.no_grad():
            for _ in range(n):
                self.f, self.g = step(self.p, self.f, self.g)
                self.t += 1
        return self

    def moments(self) -> torch.Tensor:
        with torch.no_grad():
            return totals(self.p, self.f, self.g)

    def fields(self) -> dict:
        with torch.no_grad():
            return macroscopic(self.p, self.f, self.g)

    def nusselt(self):
        with torch.no_grad():
            return nusselt(self.p, self.f, self.g)

    def state(self) -> torch.Tensor:
        return torch.cat([self.f, self.g], dim=0)
