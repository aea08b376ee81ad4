// physics.hpp - per-node arithmetic of the thermal pseudopotential D3Q19 step
// for gfx950, shared by every kernel of the library (reference, fused and
// diagnostics) so that they all compute bit-identical node updates.
//
// The scheme (arXiv:1111.0905, section "Algorithm"):
//   eq. (HYDRO)  rho = sum f, j = sum c f, E = rho T = sum g;
//   eq. (FORCE)  F_SC = -G psi(x) sum_l W_l c_l psi(x + c_l), psi = exp(-1/rho),
//                W = 1/6 (axis), 1/12 (face diagonal): isotropic to 4th order;
//   f/g coupling: f^eq carries the lattice pressure rho T_lat (constant
//                 lattice temperature, via the rest population) and the force
//                 F_T = -grad(rho T - rho T_lat) adds the rest of the ideal
//                 pressure rho T (T from the g populations);
//   gravity:      F_g = rho (0, 0, -g)  (eq. (ns));
//   velocity shift u' = (j + tau_nu F)/rho inside f^eq; physical v = (j + F/2)/rho;
//   eqs. (LBEQ)/(LBEQ2) BGK with
//     f^eq_l = w_l rho [1 + 3 c.u' + 4.5 (c.u')^2 - 1.5 u'^2] + a_l rho (T_lat - 1/3),
//       a_0 = -2, a_l = 3 w_l,
//     g^eq_l = w_l [E + gamma E (3 c.v + 4.5 (c.v)^2 - 1.5 v^2)] + b_l (rho_kappa - rho) T,
//       gamma = 1 + 1/c_v, b_0 = -2/3, b_l = w_l: one conductivity
//       kappa = c_v (tau_kappa - 1/2) rho_kappa / 3 in both phases;
//   counter-term of the g dynamics: the factor gamma plus the source
//     S = (1/c_v) v . grad E added as w_l S, so that
//     dE/dt + div(E v) = -(E/c_v) div v + (kappa/c_v) lap T (eq. (eq), 2nd form).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbm {

constexpr int Q = 19;
// D3Q19 velocity set (same order as the canonical state of the C ABI).
constexpr int CX[Q] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
constexpr int CY[Q] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
constexpr int CZ[Q] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
constexpr int OPP[Q] = {0, 2, 1, 4, 3, 6, 5, 8, 7, 10, 9, 12, 11, 14, 13, 16, 15, 18, 17};

template <typename R>
__host__ __device__ constexpr R wlat(int l) {
  return l == 0 ? R(1) / R(3) : (l < 7 ? R(1) / R(18) : R(1) / R(36));
}
// isotropic second-moment adjusters of f^eq (a) and g^eq (b)
template <typename R>
__host__ __device__ constexpr R af(int l) {
  return l == 0 ? R(-2) : R(3) * wlat<R>(l);
}
template <typename R>
__host__ __device__ constexpr R bg(int l) {
  return l == 0 ? R(-2) / R(3) : wlat<R>(l);
}

// Device-side parameters in compute precision.
template <typename R>
struct DevParams {
  int nx, ny, nz;
  int periodic_z;
  R omega_f, omega_g;   // 1/tau_nu, 1/tau_kappa
  R tau_nu;
  R G;
  R gravity;
  R inv_cv, gamma;      // 1/c_v, 1 + 1/c_v
  R rho_kappa;
  R T_d, T_u;
  R T_lat;              // lattice temperature of f^eq
  R fref[Q], gref[Q];   // deviation references (16-bit storage only)
  // psi of the ghost planes at the bottom / top wall when wet_d / wet_u
  // (prescribed wall density); otherwise the mirror image of the wall plane
  int wet_d, wet_u;
  R psi_wd, psi_wu;
  int psi_form;         // 0: exp(-1/rho); 1: 1 - exp(-rho)
};

// ----------------------------------------------------------- storage codecs
// Populations are stored in pairs: word l of a node holds (f_l, g_l), so one
// load or store moves both populations of a direction (push streaming sends
// f*_l and g*_l to the same node, also at the walls).  Stored as S, computed
// in R.  Buffer layout, structure of arrays (N nodes, node offset i):
//   FP64, FP32:  direction l at words [l N, (l + 1) N).
//   FP16, BF16:  the rest pair (l = 0) in FP32 (absolute values, N float2
//                in 32-bit words [0, 2 N)); the 18 moving directions hold
//                (pop - pop_ref) rounded to nearest even, direction l >= 1
//                at words [(l + 1) N, (l + 2) N).
// The rest population carries most of the mass (f_0 = rho (1 - 2 T_lat)),
// and in nearly uniform regions (and always for the decoded, quantised
// moving populations of the 16-bit forms) FP32 roundings of the node sums
// and of f_0 are correlated between nodes and steps and make mass drift.
// FP32 and the 16-bit forms therefore update the rest pair in remainder
// form: the new rest value is the old one plus what the 18 moving pairs gave
// up in the collision plus (16-bit forms) the rounding residuals of their
// stores, plus the energy source S for g; the small terms are accumulated in
// FP32 and added to the FP32 rest pair in Streamer::rest.  Stored mass is
// then conserved to the rounding of those sums, and the stored energy changes
// by S and the wall exchange.
struct F64 { using S = double2; using R = double; };
struct F32 { using S = float2; using R = float; };
struct H16 { using S = uint32_t; using R = float; };   // lo: f, hi: g (IEEE half)
struct B16 { using S = uint32_t; using R = float; };   // lo: f, hi: g (bfloat16)

// Wave-uniform pointer: the value is moved into scalar registers so that a
// load or store through it uses the scalar-base + 32-bit vector-offset form.
template <typename T>
__device__ __forceinline__ T* uniform_ptr(T* p) {
  const uint64_t v = (uint64_t)p;
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return (T*)(((uint64_t)hi << 32) | lo);
}

// Element i of the population array starting at p; p MUST be the same for
// every lane of the wave (it is read from the first active lane).  The byte
// offset is formed in 32 bits (the library keeps every population row
// below 4 GiB).
template <typename T>
__device__ __forceinline__ const T& at32(const T* p, uint32_t i) {
  return *(const T*)((const char*)uniform_ptr(p) + (uint32_t)(i * (uint32_t)sizeof(T)));
}
template <typename T>
__device__ __forceinline__ T& at32(T* p, uint32_t i) {
  return *(T*)((char*)uniform_ptr(p) + (uint32_t)(i * (uint32_t)sizeof(T)));
}

__device__ __forceinline__ uint32_t bf16_rne(float v) {
  uint32_t u = __builtin_bit_cast(uint32_t, v);
  u += 0x7FFFu + ((u >> 16) & 1u);   // round to nearest even (finite inputs)
  return u >> 16;
}

// Pitch of the population rows in words: the node count rounded up to a
// multiple of 16384, plus 1024.  With rows exactly 2^29 or 2^30 bytes apart
// (512^3 lattices) a stream over the 19 rows ran at 4.96 or 5.16 TB/s on
// MI355X; shifting each row by 1024 words more lifted it to 5.40 and 5.35.
__host__ __device__ constexpr size_t row_pitch(size_t N) {
  return ((N + 16383) & ~(size_t)16383) + 1024;
}

// Tile of work-group b of nb.  Work-groups are dealt round-robin over the 8
// XCDs (b on XCD b mod 8); XCD x takes a contiguous range of tiles (the first
// nb mod 8 XCDs one tile more than the others), so that neighbouring tiles
// share an L2.  A bijection of [0, nb) for every nb.
__device__ __forceinline__ int xcd_tile(int b, int nb) {
  const int x = b & 7, i = b >> 3, q = nb >> 3, r = nb & 7;
  return x < r ? x * (q + 1) + i : r * (q + 1) + (x - r) * q + i;
}

// Per storage form: enc/dec of one moving pair word, the row of direction
// l >= 1 (rows row_pitch(N) words apart), and the rest pair (type T0).  kRemainder: the rest pair is updated
// in remainder form (FP32 and the 16-bit forms); kResidual: the moving stores
// also hand their rounding residuals to it (16-bit forms).
template <typename C> struct Codec;
template <> struct Codec<F64> {
  using S = double2;
  using R = double;
  using T0 = double;
  static constexpr bool kResidual = false;
  static constexpr bool kRemainder = false;
  static __device__ __forceinline__ void dec(S w, R& f, R& g, R, R) { f = w.x; g = w.y; }
  static __device__ __forceinline__ S enc(R f, R g, R, R) { return make_double2(f, g); }
  static __device__ __forceinline__ const S* row(const S* b, int l, size_t N) {
    return b + (size_t)l * row_pitch(N);
  }
  static __device__ __forceinline__ S* row(S* b, int l, size_t N) { return b + (size_t)l * row_pitch(N); }
  static __device__ __forceinline__ void ld0(const S* b, uint32_t i, T0& f, T0& g) {
    const S w = at32(b, i);
    f = w.x;
    g = w.y;
  }
  static __device__ __forceinline__ void st0(S* b, uint32_t i, T0 f, T0 g) { at32(b, i) = make_double2(f, g); }
};
template <> struct Codec<F32> {
  using S = float2;
  using R = float;
  using T0 = float;
  static constexpr bool kResidual = false;
  static constexpr bool kRemainder = true;
  static __device__ __forceinline__ void dec(S w, R& f, R& g, R, R) { f = w.x; g = w.y; }
  static __device__ __forceinline__ S enc(R f, R g, R, R) { return make_float2(f, g); }
  static __device__ __forceinline__ const S* row(const S* b, int l, size_t N) {
    return b + (size_t)l * row_pitch(N);
  }
  static __device__ __forceinline__ S* row(S* b, int l, size_t N) { return b + (size_t)l * row_pitch(N); }
  static __device__ __forceinline__ void ld0(const S* b, uint32_t i, T0& f, T0& g) {
    const S w = at32(b, i);
    f = w.x;
    g = w.y;
  }
  static __device__ __forceinline__ void st0(S* b, uint32_t i, T0 f, T0 g) { at32(b, i) = make_float2(f, g); }
};
// The two 16-bit forms share the layout and differ in enc/dec only.
struct Dev16 {
  using S = uint32_t;
  using R = float;
  using T0 = float;
  static constexpr bool kResidual = true;
  static constexpr bool kRemainder = true;
  // the FP32 rest pair takes the first 2 N words (rows 0 and 1)
  static __device__ __forceinline__ const S* row(const S* b, int l, size_t N) {
    return b + (size_t)(l + 1) * row_pitch(N);
  }
  static __device__ __forceinline__ S* row(S* b, int l, size_t N) {
    return b + (size_t)(l + 1) * row_pitch(N);
  }
  static __device__ __forceinline__ void ld0(const S* b, uint32_t i, T0& f, T0& g) {
    const float2 w = at32((const float2*)b, i);
    f = w.x;
    g = w.y;
  }
  static __device__ __forceinline__ void st0(S* b, uint32_t i, T0 f, T0 g) {
    at32((float2*)b, i) = make_float2(f, g);
  }
};
template <> struct Codec<H16> : Dev16 {
  static __device__ __forceinline__ void dec(uint32_t u, float& f, float& g, float fr, float gr) {
    f = (float)__builtin_bit_cast(_Float16, (uint16_t)(u & 0xFFFFu)) + fr;
    g = (float)__builtin_bit_cast(_Float16, (uint16_t)(u >> 16)) + gr;
  }
  static __device__ __forceinline__ uint32_t enc(float f, float g, float fr, float gr) {
    const uint32_t lo = __builtin_bit_cast(uint16_t, (_Float16)(f - fr));
    const uint32_t hi = __builtin_bit_cast(uint16_t, (_Float16)(g - gr));
    return lo | (hi << 16);
  }
  // enc, adding (value - decoded value) to rf, rg: the decode's own FP32
  // rounding is included, and the difference of the two close floats is
  // exact, so the rest pair receives what the decoder will miss
  static __device__ __forceinline__ uint32_t enc_res(float f, float g, float fr, float gr, float& rf,
                                                     float& rg) {
    const _Float16 hf = (_Float16)(f - fr), hg = (_Float16)(g - gr);
    rf += f - ((float)hf + fr);
    rg += g - ((float)hg + gr);
    return (uint32_t)__builtin_bit_cast(uint16_t, hf) | ((uint32_t)__builtin_bit_cast(uint16_t, hg) << 16);
  }
};
template <> struct Codec<B16> : Dev16 {
  static __device__ __forceinline__ void dec(uint32_t u, float& f, float& g, float fr, float gr) {
    f = __builtin_bit_cast(float, u << 16) + fr;
    g = __builtin_bit_cast(float, u & 0xFFFF0000u) + gr;
  }
  static __device__ __forceinline__ uint32_t enc(float f, float g, float fr, float gr) {
    return bf16_rne(f - fr) | (bf16_rne(g - gr) << 16);
  }
  static __device__ __forceinline__ uint32_t enc_res(float f, float g, float fr, float gr, float& rf,
                                                     float& rg) {
    const uint32_t uf = bf16_rne(f - fr), ug = bf16_rne(g - gr);
    rf += f - (__builtin_bit_cast(float, uf << 16) + fr);
    rg += g - (__builtin_bit_cast(float, ug << 16) + gr);
    return uf | (ug << 16);
  }
};

// Load the pair of direction l (any l) of node i, in the compute type.
template <typename C, typename R = typename C::R>
__device__ __forceinline__ void load_pair(const typename C::S* b, int l, size_t N, uint32_t i, R& f,
                                          R& g, R fr, R gr) {
  if (l == 0) {
    typename Codec<C>::T0 f0, g0;
    Codec<C>::ld0(b, i, f0, g0);
    f = (R)f0;
    g = (R)g0;
  } else {
    Codec<C>::dec(at32(Codec<C>::row(b, l, N), i), f, g, fr, gr);
  }
}

// Store the pair of a moving direction l >= 1 of node i; with kResidual the
// rounding residuals (value - stored value) are added to rf, rg.
template <typename C, typename R = typename C::R>
__device__ __forceinline__ void store_moving(typename C::S* b, int l, size_t N, uint32_t i, R f, R g,
                                             R fr, R gr, R& rf, R& rg) {
  if constexpr (Codec<C>::kResidual)
    at32(Codec<C>::row(b, l, N), i) = Codec<C>::enc_res(f, g, fr, gr, rf, rg);
  else
    at32(Codec<C>::row(b, l, N), i) = Codec<C>::enc(f, g, fr, gr);
}

// ----------------------------------------------------------- node arithmetic

template <typename R>
__device__ __forceinline__ R psi_of(R rho, int form) {
  // one exponential for either form (form is uniform over the launch)
  const R e = exp(form ? -rho : R(-1) / rho);
  return form ? R(1) - e : e;
}

// W-stencil central gradient sum_l W_l c_l a(x + c_l); at(l) returns the
// neighbour value in direction l.
template <typename R, typename A>
__device__ __forceinline__ void grad_w(const A& at, R& gx, R& gy, R& gz) {
  const R a1 = at(1), a2 = at(2), a3 = at(3), a4 = at(4), a5 = at(5), a6 = at(6);
  const R a7 = at(7), a8 = at(8), a9 = at(9), a10 = at(10), a11 = at(11), a12 = at(12);
  const R a13 = at(13), a14 = at(14), a15 = at(15), a16 = at(16), a17 = at(17), a18 = at(18);
  const R s6 = R(1) / R(6), s12 = R(1) / R(12);
  gx = s6 * (a1 - a2) + s12 * (((a7 - a8) + (a9 - a10)) + ((a11 - a12) + (a13 - a14)));
  gy = s6 * (a3 - a4) + s12 * (((a7 - a8) - (a9 - a10)) + ((a15 - a16) + (a17 - a18)));
  gz = s6 * (a5 - a6) + s12 * (((a11 - a12) - (a13 - a14)) + ((a15 - a16) - (a17 - a18)));
}

template <typename R>
struct Macro {
  R rho, E, T, psi;
  R jx, jy, jz;
  R Fx, Fy, Fz;
  R vx, vy, vz;   // physical velocity (j + F/2)/rho
  R S;            // counter-term source (1/c_v) v . grad E
};

template <typename R>
__device__ __forceinline__ void moments(const R* f, const R* g, R& rho, R& E) {
  R r = R(0), e = R(0);
#pragma unroll
  for (int l = 0; l < Q; ++l) { r += f[l]; e += g[l]; }
  rho = r;
  E = e;
}

// Momentum sum_l c_l f_l of a node's populations.
template <typename R>
__device__ __forceinline__ void momentum(const R* f, R& jx, R& jy, R& jz) {
  jx = ((f[1] - f[2]) + (f[7] - f[8])) + ((f[9] - f[10]) + (f[11] - f[12])) + (f[13] - f[14]);
  jy = ((f[3] - f[4]) + (f[7] - f[8])) + ((f[10] - f[9]) + (f[15] - f[16])) + (f[17] - f[18]);
  jz = ((f[5] - f[6]) + (f[11] - f[12])) + ((f[14] - f[13]) + (f[15] - f[16])) + (f[18] - f[17]);
}

// Node-local macroscopic quantities from the node's moments (rho, E,
// momentum j) and the three neighbour gradients (psi, E, rho).
template <typename R>
__device__ __forceinline__ Macro<R> node_macro(R jx, R jy, R jz, R rho, R E, R psi,
                                               R gpx, R gpy, R gpz, R gEx, R gEy, R gEz,
                                               R grx, R gry, R grz, const DevParams<R>& P) {
  Macro<R> m;
  m.rho = rho;
  m.E = E;
  m.psi = psi;
  m.T = E / rho;
  m.jx = jx;
  m.jy = jy;
  m.jz = jz;
  const R gp = -P.G * psi;
  m.Fx = gp * gpx - (gEx - P.T_lat * grx);
  m.Fy = gp * gpy - (gEy - P.T_lat * gry);
  m.Fz = gp * gpz - (gEz - P.T_lat * grz) - P.gravity * rho;
  const R ir = R(1) / rho;
  m.vx = (m.jx + R(0.5) * m.Fx) * ir;
  m.vy = (m.jy + R(0.5) * m.Fy) * ir;
  m.vz = (m.jz + R(0.5) * m.Fz) * ir;
  m.S = (m.vx * gEx + m.vy * gEy + m.vz * gEz) * P.inv_cv;
  return m;
}

template <typename R>
__device__ __forceinline__ Macro<R> node_macro(const R* f, const R* g, R rho, R E, R psi,
                                               R gpx, R gpy, R gpz, R gEx, R gEy, R gEz,
                                               R grx, R gry, R grz, const DevParams<R>& P) {
  R jx, jy, jz;
  momentum<R>(f, jx, jy, jz);
  return node_macro<R>(jx, jy, jz, rho, E, psi, gpx, gpy, gpz, gEx, gEy, gEz, grx, gry, grz, P);
}

// BGK collision of both populations at one node (eqs. (LBEQ)/(LBEQ2) right
// hand sides plus the counter-term).  emit(l, f*_l, g*_l, df_l, dg_l)
// receives the collided values of the moving directions and what the
// collision took from them; emit.rest(f*_0, g*_0, S) the rest pair, last.
template <typename R, typename Emit>
__device__ __forceinline__ void collide(const R* f, const R* g, const Macro<R>& m,
                                        const DevParams<R>& P, Emit&& emit) {
  const R ir = R(1) / m.rho;
  const R ux = (m.jx + P.tau_nu * m.Fx) * ir;
  const R uy = (m.jy + P.tau_nu * m.Fy) * ir;
  const R uz = (m.jz + P.tau_nu * m.Fz) * ir;
  const R uu = R(1) - R(1.5) * (ux * ux + uy * uy + uz * uz);
  const R vv = R(-1.5) * (m.vx * m.vx + m.vy * m.vy + m.vz * m.vz);
  const R gE = P.gamma * m.E;
  const R rk = (P.rho_kappa - m.rho) * m.T;
  const R rt = m.rho * (P.T_lat - R(1) / R(3));
#pragma unroll
  for (int q = 1; q <= Q; ++q) {
    const int l = q == Q ? 0 : q;
    const R cu = R(CX[l]) * ux + R(CY[l]) * uy + R(CZ[l]) * uz;
    const R cv = R(CX[l]) * m.vx + R(CY[l]) * m.vy + R(CZ[l]) * m.vz;
    const R w = wlat<R>(l);
    const R feq = w * m.rho * (uu + cu * (R(3) + R(4.5) * cu)) + af<R>(l) * rt;
    const R geq = w * (m.E + gE * (vv + cv * (R(3) + R(4.5) * cv))) + bg<R>(l) * rk;
    // what the pair gives up in the collision, and the collided values
    const R df = P.omega_f * (f[l] - feq);
    const R dg = P.omega_g * (g[l] - geq) - w * m.S;
    const R fs = f[l] - df;
    const R gs = g[l] - dg;
    if (l == 0)
      emit.rest(fs, gs, m.S);
    else
      emit(l, fs, gs, df, dg);
  }
}

// Local equilibrium at rest (initial state).
template <typename R>
__device__ __forceinline__ void rest_equilibrium(R rho, R T, R rho_kappa, R T_lat, R* f, R* g) {
  const R E = rho * T;
  const R rk = (rho_kappa - rho) * T;
  const R rt = rho * (T_lat - R(1) / R(3));
#pragma unroll
  for (int l = 0; l < Q; ++l) {
    f[l] = wlat<R>(l) * rho + af<R>(l) * rt;
    g[l] = wlat<R>(l) * E + bg<R>(l) * rk;
  }
}

}  // namespace lbm
