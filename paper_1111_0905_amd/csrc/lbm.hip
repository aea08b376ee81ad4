// lbm.hip - HIP kernels (gfx950) and the C ABI of the thermal pseudopotential
// D3Q19 lattice Boltzmann step (arXiv:1111.0905, section "Algorithm").
// The ABI is declared and documented in include/lbm.h.
//
// Data layout in HBM: structure of arrays of pairs: word l of node (i, j, k)
// holds (f_l, g_l) at l * N + (k * ny + j) * nx + i (i fastest) for FP64 and
// FP32; the 16-bit forms keep the rest pair in FP32 ahead of the 18 moving
// rows (see the codecs in physics.hpp); two
// ping-pong buffers hold the post-streaming populations.  Streaming is a push: the collided value of
// node x in direction l is written to x + c_l of the other buffer; at the
// walls it is written back to x in direction opp(l) (half-way bounce-back for
// f, anti-bounce-back about w_l rho_kappa T_wall for g).
//
// Kernels
//   k_fused      one launch per step: a work-group owns a 64 x TY column of
//                the x-y plane and marches up a chunk of z planes; rho, E and
//                psi of the current plane and its two neighbours (tile plus a
//                one-node ring) sit in an LDS ring buffer, so every population
//                is read from HBM once and written once per step.
//   k_rhoE +     reference two-pass step (and the diagnostics): rho and E of
//   k_collide    every node to scratch, then collide+stream per node.
//   k_diag, k_plane, k_finish_*   FP64 reductions for the diagnostics.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <new>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/lbm.h"
#include "physics.hpp"

using namespace lbm;

namespace {

thread_local std::string g_err;

// Scratch of the allocation-free entry point (lbm_structure_functions_noalloc):
// one array per GPU the library runs on, held until the process ends.  Host
// code never uses the array's name as an address: lbm_init takes each
// device's address once with hipGetSymbolAddress and keeps it per device.
constexpr size_t kStaticScratchDoubles = (size_t)4 << 20;   // 32 MiB
__device__ __align__(256) double scratch[kStaticScratchDoubles];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

#define HIP_TRY(expr)                                                              \
  do {                                                                             \
    hipError_t e_ = (expr);                                                        \
    if (e_ != hipSuccess)                                                          \
      return fail(LBM_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_));    \
  } while (0)

// 32-bit node offset (the library limits N to < 2^31 nodes).
__device__ __forceinline__ uint32_t node_off(int i, int j, int k, int nx, int ny) {
  return ((uint32_t)k * (uint32_t)ny + (uint32_t)j) * (uint32_t)nx + (uint32_t)i;
}
__device__ __forceinline__ int wrap(int a, int n) { return a < 0 ? a + n : (a >= n ? a - n : a); }

// Push-stream the collided values of node (i, j, k) into `out`: operator()
// for the moving directions, then rest() for the rest pair, which stays at
// the node.
template <typename C, typename R = typename C::R>
struct Streamer {
  using T0 = typename Codec<C>::T0;
  typename C::S* out;
  const typename C::S* in;   // this step's input (the rest pair is re-read from it)
  const DevParams<R>& P;
  size_t N;
  int i, j, k, im, ip, jm, jp;
  // what the moving pairs gave up: the collision increments plus (stored
  // value - decoded stored value), summed over the 18 directions
  R rf = R(0), rg = R(0);
  // fs, gs: collided values of direction l; df, dg: what the collision took
  // from the pair (f_l - fs up to the rounding of fs)
  __device__ __forceinline__ void operator()(int l, R fs, R gs, R df, R dg) {
    if constexpr (Codec<C>::kRemainder) {
      rf += df;
      rg += dg;
    }
    const int nz = P.nz;
    int kk = k + CZ[l];
    const int ii = CX[l] > 0 ? ip : (CX[l] < 0 ? im : i);
    const int jj = CY[l] > 0 ? jp : (CY[l] < 0 ? jm : j);
    if (kk >= 0 && kk < nz) {
      store_moving<C>(out, l, N, node_off(ii, jj, kk, P.nx, P.ny), fs, gs, P.fref[l], P.gref[l],
                      rf, rg);
    } else if (P.periodic_z) {
      kk = kk < 0 ? kk + nz : kk - nz;
      store_moving<C>(out, l, N, node_off(ii, jj, kk, P.nx, P.ny), fs, gs, P.fref[l], P.gref[l],
                      rf, rg);
    } else {  // the wall sends it back into this node in the opposite direction
      const R Tw = kk < 0 ? P.T_d : P.T_u;
      const int q = OPP[l];
      store_moving<C>(out, q, N, node_off(i, j, k, P.nx, P.ny), fs,
                      -gs + R(2) * wlat<R>(l) * P.rho_kappa * Tw, P.fref[q], P.gref[q], rf, rg);
    }
  }
  // fs, gs: the BGK values of the rest pair; S: the node's energy source
  __device__ __forceinline__ void rest(R fs, R gs, R S) {
    const uint32_t o = node_off(i, j, k, P.nx, P.ny);
    if constexpr (Codec<C>::kRemainder) {  // remainder form: mass kept, energy + S
      T0 f0, g0;
      Codec<C>::ld0(in, o, f0, g0);
      Codec<C>::st0(out, o, f0 + (T0)rf, g0 + (T0)(S + rg));
    } else {
      Codec<C>::st0(out, o, fs, gs);
    }
  }
};

template <typename C, typename R = typename C::R>
__device__ __forceinline__ void load_node(const typename C::S* __restrict__ in, size_t N, uint32_t o,
                                          const DevParams<R>& P, R* f, R* g) {
#pragma unroll
  for (int l = 0; l < Q; ++l) load_pair<C>(in, l, N, o, f[l], g[l], P.fref[l], P.gref[l]);
}

// Store all pairs of node o in place (no streaming) from FP64 values; the
// 16-bit forms add the rounding residuals of the moving pairs (taken in FP64)
// to the rest pair, so the stored sums equal the given ones.
template <typename C, typename R = typename C::R>
__device__ __forceinline__ void store_node(typename C::S* out, size_t N, uint32_t o,
                                           const DevParams<R>& P, const double* f, const double* g) {
  using T0 = typename Codec<C>::T0;
  double rf = 0.0, rg = 0.0;
#pragma unroll
  for (int l = 1; l < Q; ++l) {
    const typename C::S w = Codec<C>::enc((R)f[l], (R)g[l], P.fref[l], P.gref[l]);
    at32(Codec<C>::row(out, l, N), o) = w;
    if constexpr (Codec<C>::kResidual) {
      R fd, gd;
      Codec<C>::dec(w, fd, gd, P.fref[l], P.gref[l]);
      rf += f[l] - (double)fd;
      rg += g[l] - (double)gd;
    }
  }
  Codec<C>::st0(out, o, (T0)(f[0] + rf), (T0)(g[0] + rg));
}

// ---------------------------------------------------------------- init / state

template <typename C, typename R = typename C::R>
__global__ void k_init(typename C::S* out, const double* __restrict__ rho0,
                       const double* __restrict__ T0, DevParams<R> P) {
  const size_t N = (size_t)P.nx * P.ny * P.nz;
  for (size_t n = blockIdx.x * (size_t)blockDim.x + threadIdx.x; n < N;
       n += (size_t)gridDim.x * blockDim.x) {
    const int k = (int)(n / ((size_t)P.nx * P.ny));
    R T;
    if (T0) {
      T = (R)T0[n];
    } else {  // conduction profile between the half-way walls
      T = (R)((double)P.T_d + ((double)P.T_u - (double)P.T_d) * ((double)k + 0.5) / (double)P.nz);
    }
    double f[Q], g[Q];
    rest_equilibrium<double>(rho0[n], (double)T, (double)P.rho_kappa, (double)P.T_lat, f, g);
    store_node<C>(out, N, (uint32_t)n, P, f, g);
  }
}

// Seeded initial density rho_mean (1 + a (2u - 1)), u the top 53 bits of
// SplitMix64 (Steele, Lea and Flood, OOPSLA 2014) evaluated at state
// seed + (n + 1) * 0x9E3779B97F4A7C15 for node counter n = i + nx (j + ny k),
// divided by 2^53.  The arithmetic is IEEE double, each operation rounded
// on its own (contraction off), so the field equals any other
// implementation of the same definition bit for bit.
__global__ void k_seeded_density(double* __restrict__ out, size_t N, uint64_t seed,
                                 double rho_mean, double amp) {
#pragma clang fp contract(off)
  for (size_t n = blockIdx.x * (size_t)blockDim.x + threadIdx.x; n < N;
       n += (size_t)gridDim.x * blockDim.x) {
    uint64_t z = seed + ((uint64_t)n + 1ull) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z = z ^ (z >> 31);
    const double u = (double)(z >> 11) * (1.0 / 9007199254740992.0);
    const double t = 2.0 * u - 1.0;
    out[n] = rho_mean * (1.0 + amp * t);
  }
}

template <typename C, typename R = typename C::R>
__global__ void k_get_state(const typename C::S* __restrict__ in, double* __restrict__ st,
                            DevParams<R> P) {
  const size_t N = (size_t)P.nx * P.ny * P.nz;
  for (size_t n = blockIdx.x * (size_t)blockDim.x + threadIdx.x; n < N;
       n += (size_t)gridDim.x * blockDim.x) {
    R f[Q], g[Q];
    load_node<C>(in, N, (uint32_t)n, P, f, g);
    typename Codec<C>::T0 f0, g0;
    Codec<C>::ld0(in, (uint32_t)n, f0, g0);
    st[n] = (double)f0;
    st[(size_t)Q * N + n] = (double)g0;
#pragma unroll
    for (int l = 1; l < Q; ++l) {
      st[(size_t)l * N + n] = (double)f[l];
      st[(size_t)(l + Q) * N + n] = (double)g[l];
    }
  }
}

template <typename C, typename R = typename C::R>
__global__ void k_set_state(typename C::S* out, const double* __restrict__ st, DevParams<R> P) {
  const size_t N = (size_t)P.nx * P.ny * P.nz;
  for (size_t n = blockIdx.x * (size_t)blockDim.x + threadIdx.x; n < N;
       n += (size_t)gridDim.x * blockDim.x) {
    double f[Q], g[Q];
#pragma unroll
    for (int l = 0; l < Q; ++l) {
      f[l] = st[(size_t)l * N + n];
      g[l] = st[(size_t)(l + Q) * N + n];
    }
    store_node<C>(out, N, (uint32_t)n, P, f, g);
  }
}

// ---------------------------------------------------------------- reference path

// rho and E of every node into scratch.
template <typename C, typename R = typename C::R>
__global__ void k_rhoE(const typename C::S* __restrict__ in, R* __restrict__ srho,
                       R* __restrict__ sE, R* __restrict__ spsi, DevParams<R> P) {
  const size_t N = (size_t)P.nx * P.ny * P.nz;
  for (size_t n = blockIdx.x * (size_t)blockDim.x + threadIdx.x; n < N;
       n += (size_t)gridDim.x * blockDim.x) {
    R f[Q], g[Q];
    load_node<C>(in, N, (uint32_t)n, P, f, g);
    R rho, E;
    moments<R>(f, g, rho, E);
    srho[n] = rho;
    sE[n] = E;
    spsi[n] = psi_of<R>(rho, P.psi_form);
  }
}

// Neighbour values from scratch with the wall ghosts: psi from the mirrored
// density (or the prescribed wall density), rho and E extrapolated linearly
// through the wall.  spsi: psi of every node (written with rho and E), or
// NULL to evaluate psi from rho here.
template <typename R>
struct ScratchNb {
  const R* srho;
  const R* sE;
  const DevParams<R>& P;
  int i, j, k;
  const R* spsi = nullptr;
  // which: 0 = psi, 1 = rho, 2 = E
  __device__ __forceinline__ R get(int which, int l) const {
    const int nx = P.nx, ny = P.ny, nz = P.nz;
    const int ii = wrap(i + CX[l], nx), jj = wrap(j + CY[l], ny);
    int kk = k + CZ[l];
    const R* a = which == 2 ? sE : srho;
    if (kk >= 0 && kk < nz) {
      const uint32_t o = node_off(ii, jj, kk, nx, ny);
      if (which == 0 && spsi) return spsi[o];
      const R v = a[o];
      return which == 0 ? psi_of<R>(v, P.psi_form) : v;
    }
    if (P.periodic_z) {
      kk = kk < 0 ? kk + nz : kk - nz;
      const uint32_t o = node_off(ii, jj, kk, nx, ny);
      if (which == 0 && spsi) return spsi[o];
      const R v = a[o];
      return which == 0 ? psi_of<R>(v, P.psi_form) : v;
    }
    const int kw = kk < 0 ? 0 : nz - 1;     // wall plane
    const int ki = kk < 0 ? 1 : nz - 2;     // next plane inside
    if (which == 0 && (kk < 0 ? P.wet_d : P.wet_u)) return kk < 0 ? P.psi_wd : P.psi_wu;
    if (which == 0 && spsi) return spsi[node_off(ii, jj, kw, nx, ny)];
    const R v0 = a[node_off(ii, jj, kw, nx, ny)];
    if (which == 0) return psi_of<R>(v0, P.psi_form);
    const R v1 = a[node_off(ii, jj, ki, nx, ny)];
    return R(2) * v0 - v1;
  }
  // psi, rho and E of neighbour l at once (one address computation)
  __device__ __forceinline__ void get3(int l, R& psi, R& rho, R& E) const {
    const int nx = P.nx, ny = P.ny, nz = P.nz;
    const int ii = wrap(i + CX[l], nx), jj = wrap(j + CY[l], ny);
    int kk = k + CZ[l];
    if ((kk >= 0 && kk < nz) || P.periodic_z) {
      kk = kk < 0 ? kk + nz : (kk >= nz ? kk - nz : kk);
      const size_t o = node_off(ii, jj, kk, nx, ny);
      rho = srho[o];
      E = sE[o];
      psi = spsi ? spsi[o] : psi_of<R>(rho, P.psi_form);
      return;
    }
    const int kw = kk < 0 ? 0 : nz - 1;     // wall plane
    const int ki = kk < 0 ? 1 : nz - 2;     // next plane inside
    const size_t ow = node_off(ii, jj, kw, nx, ny), oi = node_off(ii, jj, ki, nx, ny);
    const R r0 = srho[ow];
    rho = R(2) * r0 - srho[oi];
    E = R(2) * sE[ow] - sE[oi];
    psi = (kk < 0 ? P.wet_d : P.wet_u) ? (kk < 0 ? P.psi_wd : P.psi_wu)
                                       : (spsi ? spsi[ow] : psi_of<R>(r0, P.psi_form));
  }
};

template <typename R>
__device__ __forceinline__ Macro<R> macro_from_scratch(const R* f, const R* g, const ScratchNb<R>& nb,
                                                       const DevParams<R>& P) {
  R rho, E;
  moments<R>(f, g, rho, E);
  R gpx, gpy, gpz, gEx, gEy, gEz, grx, gry, grz;
  R pn[Q], rn[Q], en[Q];
#pragma unroll
  for (int l = 1; l < Q; ++l) nb.get3(l, pn[l], rn[l], en[l]);
  grad_w<R>([&](int l) { return pn[l]; }, gpx, gpy, gpz);
  grad_w<R>([&](int l) { return en[l]; }, gEx, gEy, gEz);
  grad_w<R>([&](int l) { return rn[l]; }, grx, gry, grz);
  return node_macro<R>(f, g, rho, E, psi_of<R>(rho, P.psi_form), gpx, gpy, gpz, gEx, gEy, gEz, grx, gry, grz, P);
}

template <typename C, typename R = typename C::R>
__global__ void k_collide(const typename C::S* __restrict__ in, typename C::S* __restrict__ out,
                          const R* __restrict__ srho, const R* __restrict__ sE,
                          const R* __restrict__ spsi, DevParams<R> P) {
  const size_t N = (size_t)P.nx * P.ny * P.nz;
  for (size_t n = blockIdx.x * (size_t)blockDim.x + threadIdx.x; n < N;
       n += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(n % P.nx);
    const int j = (int)((n / P.nx) % P.ny);
    const int k = (int)(n / ((size_t)P.nx * P.ny));
    R f[Q], g[Q];
    load_node<C>(in, N, (uint32_t)n, P, f, g);
    ScratchNb<R> nb{srho, sE, P, i, j, k, spsi};
    const Macro<R> m = macro_from_scratch<R>(f, g, nb, P);
    Streamer<C> em{out, in, P, N, i, j, k, wrap(i - 1, P.nx), wrap(i + 1, P.nx),
                   wrap(j - 1, P.ny), wrap(j + 1, P.ny)};
    collide<R>(f, g, m, P, em);
  }
}

// ---------------------------------------------------------------- fused path

// One work-group: tile of TX x TY nodes in x-y, planes [k0, k1) in z.
// LDS ring buffer of four plane slots of psi, rho and E over the tile plus a
// one-node ring; the populations of the plane being collided and of the next
// plane are held in registers, so each population is read once from HBM.
template <typename C, int TX, int TY, bool KEEP, typename R = typename C::R>
__global__ __launch_bounds__(TX * TY) void k_fused(const typename C::S* __restrict__ in,
                                                  typename C::S* __restrict__ out,
                                                  DevParams<R> P, int ntx, int nty, int kz) {
  constexpr int PW = TX + 2, PN = PW * (TY + 2);
  // four plane slots: the plane written by fill(k+1) was last read by
  // collide(k-2), so a single barrier per plane separates writers and readers
  constexpr int NS = 4;
  __shared__ R sPsi[NS][PN];
  __shared__ R sRho[NS][PN];
  __shared__ R sE[NS][PN];

  const int nx = P.nx, ny = P.ny, nz = P.nz;
  const size_t N = (size_t)nx * ny * nz;

  // XCD-aware tile order: consecutive tiles land on the same XCD (work-groups
  // are dealt round-robin over the 8 XCDs), so neighbouring tiles share L2.
  const int bid = xcd_tile(blockIdx.x, gridDim.x);
  const int tx = bid % ntx;
  const int rem = bid / ntx;
  const int ty = rem % nty;
  const int zc = rem / nty;
  const int x0 = tx * TX, y0 = ty * TY;
  const int k0 = zc * kz;
  const int k1 = min(k0 + kz, nz);
  const int tw = min(TX, nx - x0), th = min(TY, ny - y0);

  const int t = threadIdx.x;
  const int lx = t % TX, ly = t / TX;
  const bool active = lx < tw && ly < th;
  const int i = x0 + lx, j = y0 + ly;
  const int im = wrap(i - 1, nx), ip = wrap(i + 1, nx), jm = wrap(j - 1, ny), jp = wrap(j + 1, ny);
  const int own_s = (ly + 1) * PW + (lx + 1);

  // the one-node ring around the tile: 2 (tw + 2) + 2 th nodes, dealt to the
  // threads in turn
  constexpr int NT = TX * TY;
  const int nring = 2 * (tw + 2) + 2 * th;
  auto ring_xy = [&](int r, int& rx, int& ry) {
    if (r < tw + 2) {
      rx = r - 1;
      ry = -1;
    } else if (r < 2 * (tw + 2)) {
      rx = r - (tw + 2) - 1;
      ry = th;
    } else {
      const int q = r - 2 * (tw + 2);
      rx = q < th ? -1 : tw;
      ry = q < th ? q : q - th;
    }
  };

  auto slot = [&](int kp) { return (kp - k0 + NS) % NS; };

  // rho, E, psi of plane kp (global index, already wrapped) into LDS slot s;
  // the own populations are left in f, g when KEEP (else they are reloaded
  // from cache when the plane is collided).
  using S = typename C::S;
  // the own node's stored words of plane kp go to w (KEEP) and are decoded
  // again when the plane is collided; this keeps the 16-bit forms packed
  using T0 = typename Codec<C>::T0;
  auto fill = [&](int kp, int s, S* w, T0& w0f, T0& w0g) {
    if (active) {
      const uint32_t o = node_off(i, j, kp, nx, ny);
      T0 f0, g0;
      Codec<C>::ld0(in, o, f0, g0);
      if (KEEP) {
        w0f = f0;
        w0g = g0;
      }
      R rho = (R)f0, E = (R)g0;
#pragma unroll
      for (int l = 1; l < Q; ++l) {
        const S v = at32(Codec<C>::row(in, l, N), o);
        if (KEEP) w[l] = v;
        R f, g;
        Codec<C>::dec(v, f, g, P.fref[l], P.gref[l]);
        rho += f;
        E += g;
      }
      sRho[s][own_s] = rho;
      sE[s][own_s] = E;
      sPsi[s][own_s] = psi_of<R>(rho, P.psi_form);
    }
    for (int r = t; r < nring; r += NT) {
      int rx, ry;
      ring_xy(r, rx, ry);
      const int ring_s = (ry + 1) * PW + (rx + 1);
      R fr[Q], gr[Q];
      load_node<C>(in, N, node_off(wrap(x0 + rx, nx), wrap(y0 + ry, ny), kp, nx, ny), P, fr, gr);
      R rho, E;
      moments<R>(fr, gr, rho, E);
      sRho[s][ring_s] = rho;
      sE[s][ring_s] = E;
      sPsi[s][ring_s] = psi_of<R>(rho, P.psi_form);
    }
  };
  // wall ghost plane: psi mirrored (or that of the prescribed wall density),
  // rho and E extrapolated linearly
  auto ghost = [&](int sg, int sw, int si, int wet, R psi_w) {
    for (int q = t; q < PN; q += NT) {
      sPsi[sg][q] = wet ? psi_w : sPsi[sw][q];
      sRho[sg][q] = R(2) * sRho[sw][q] - sRho[si][q];
      sE[sg][q] = R(2) * sE[sw][q] - sE[si][q];
    }
  };

  S wa[Q], wb[Q];             // raw words of the moving pairs (KEEP); [0] unused
  T0 wa0f, wa0g, wb0f, wb0g;  // the rest pair (KEEP)
  const bool walls = !P.periodic_z;
  if (k0 > 0)
    fill(k0 - 1, slot(k0 - 1), wb, wb0f, wb0g);
  else if (!walls)
    fill(nz - 1, slot(k0 - 1), wb, wb0f, wb0g);
  fill(k0, slot(k0), wa, wa0f, wa0g);

  for (int k = k0; k < k1; ++k) {
    const int kn = k + 1;
    if (kn < nz)
      fill(kn, slot(kn), wb, wb0f, wb0g);
    else if (!walls)
      fill(0, slot(kn), wb, wb0f, wb0g);
    __syncthreads();
    if (walls && (k == 0 || kn == nz)) {
      if (k == 0) ghost(slot(-1), slot(0), slot(1), P.wet_d, P.psi_wd);
      if (kn == nz) ghost(slot(kn), slot(k), slot(k - 1), P.wet_u, P.psi_wu);
      __syncthreads();
    }
    if (active) {
      R fa[Q], ga[Q];
      T0 f0, g0;
      if (KEEP) {
        f0 = wa0f;
        g0 = wa0g;
#pragma unroll
        for (int l = 1; l < Q; ++l) Codec<C>::dec(wa[l], fa[l], ga[l], P.fref[l], P.gref[l]);
      } else {
        const uint32_t o = node_off(i, j, k, nx, ny);
        Codec<C>::ld0(in, o, f0, g0);
#pragma unroll
        for (int l = 1; l < Q; ++l) load_pair<C>(in, l, N, o, fa[l], ga[l], P.fref[l], P.gref[l]);
      }
      fa[0] = (R)f0;
      ga[0] = (R)g0;
      const int sm = slot(k - 1), s0 = slot(k), sp = slot(k + 1);
      auto at = [&](const R(*A)[PN], int l) {
        const int s = CZ[l] < 0 ? sm : (CZ[l] > 0 ? sp : s0);
        return A[s][own_s + CY[l] * PW + CX[l]];
      };
      R gpx, gpy, gpz, gEx, gEy, gEz, grx, gry, grz;
      grad_w<R>([&](int l) { return at(sPsi, l); }, gpx, gpy, gpz);
      grad_w<R>([&](int l) { return at(sE, l); }, gEx, gEy, gEz);
      grad_w<R>([&](int l) { return at(sRho, l); }, grx, gry, grz);
      const Macro<R> m = node_macro<R>(fa, ga, sRho[s0][own_s], sE[s0][own_s], sPsi[s0][own_s],
                                       gpx, gpy, gpz, gEx, gEy, gEz, grx, gry, grz, P);
      Streamer<C> em{out, in, P, N, i, j, k, im, ip, jm, jp};
      collide<R>(fa, ga, m, P, em);
    }
    if (KEEP) {
      wa0f = wb0f;
      wa0g = wb0g;
#pragma unroll
      for (int l = 1; l < Q; ++l) wa[l] = wb[l];
    }
  }
}

// ---------------------------------------------------------------- pipelined path

#include "pipe.hpp"

// ---------------------------------------------------------------- bandwidth references

#include "probe.hpp"

// ---------------------------------------------------------------- diagnostics

__device__ __forceinline__ double block_sum(double v, double* sh) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  const int w = threadIdx.x / 64, lane = threadIdx.x % 64;
  __syncthreads();
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int q = 0; q < (int)(blockDim.x / 64); ++q) s += sh[q];
  return s;  // valid in thread 0
}

// Per node: fields (optional) and block partial sums of
// [rho, rho vx, rho vy, rho vz, rho T, rho U, #bad].
template <typename C, typename R = typename C::R>
__global__ __launch_bounds__(256) void k_diag(const typename C::S* __restrict__ in,
                                              const R* __restrict__ srho, const R* __restrict__ sE,
                                              const R* __restrict__ spsi,
                                              DevParams<R> P, double c_v, double G,
                                              double* __restrict__ fields,
                                              double* __restrict__ partials) {
  __shared__ double sh[4];
  const size_t N = (size_t)P.nx * P.ny * P.nz;
  double acc[7] = {0, 0, 0, 0, 0, 0, 0};
  // node indices fit 32 bits (every population row stays below 4 GiB)
  const uint32_t N32 = (uint32_t)N, nx = (uint32_t)P.nx, ny = (uint32_t)P.ny;
  for (uint32_t n = blockIdx.x * blockDim.x + threadIdx.x; n < N32; n += gridDim.x * blockDim.x) {
    const uint32_t r = n / nx;
    const int i = (int)(n - r * nx);
    const int j = (int)(r % ny);
    const int k = (int)(r / ny);
    R f[Q], g[Q];
    load_node<C>(in, N, (uint32_t)n, P, f, g);
    ScratchNb<R> nb{srho, sE, P, i, j, k, spsi};
    const Macro<R> m = macro_from_scratch<R>(f, g, nb, P);
    // mass and energy sums of the stored populations in FP64 (the FP32 node
    // sums of the compute path round the same way at nodes of equal state,
    // which would bias a global sum)
    typename Codec<C>::T0 f0, g0;
    Codec<C>::ld0(in, (uint32_t)n, f0, g0);
    double rho = (double)f0, E = (double)g0;
#pragma unroll
    for (int l = 1; l < Q; ++l) {
      rho += (double)f[l];
      E += (double)g[l];
    }
    const double T = E / rho;
    const double U = c_v * T + 0.25 * G * exp(-2.0 / rho);
    acc[0] += rho;
    acc[1] += rho * (double)m.vx;
    acc[2] += rho * (double)m.vy;
    acc[3] += rho * (double)m.vz;
    acc[4] += E;
    acc[5] += rho * U;
    const bool bad = !(rho > 0.0) || !isfinite(rho) || !isfinite(T) || !isfinite((double)m.vx) ||
                     !isfinite((double)m.vy) || !isfinite((double)m.vz);
    acc[6] += bad ? 1.0 : 0.0;
    if (fields) {
      fields[n] = rho;
      fields[N + n] = m.vx;
      fields[2 * N + n] = m.vy;
      fields[3 * N + n] = m.vz;
      fields[4 * N + n] = T;
    }
  }
  for (int q = 0; q < 7; ++q) {
    const double s = block_sum(acc[q], sh);
    if (threadIdx.x == 0) partials[(size_t)blockIdx.x * 8 + q] = s;
  }
}

// Histogram of node quantities over planes [k0, k1) (joint histogram of two
// quantities, or of one when qy < 0), plus FP64 block partial sums
// [count, sum x, sum x^2, sum y, sum y^2, out of range].  A node falls in bin
// (floor((x - xlo) * xscale), floor((y - ylo) * yscale)) when both lie in
// [0, nbins); x, y in FP64 from the FP64 node sums.  Bins are counted in LDS
// (nbins <= kLdsBins) or straight into `counts`.
struct HistSpec {
  int k0, k1, qx, qy, nxb, nyb;
  double xlo, xscale, ylo, yscale;
};
constexpr int kLdsBins = 16384;

template <typename C, typename R = typename C::R>
__global__ __launch_bounds__(256) void k_hist(const typename C::S* __restrict__ in,
                                              const R* __restrict__ srho, const R* __restrict__ sE,
                                              const R* __restrict__ spsi,
                                              DevParams<R> P, double c_v, double G, HistSpec hs,
                                              unsigned long long* __restrict__ counts,
                                              double* __restrict__ partials) {
  extern __shared__ uint32_t sh_bins[];
  __shared__ double sh[4];
  const int nbins = hs.nxb * hs.nyb;
  const bool lds = nbins <= kLdsBins;
  if (lds)
    for (int q = threadIdx.x; q < nbins; q += blockDim.x) sh_bins[q] = 0u;
  __syncthreads();
  const size_t N = (size_t)P.nx * P.ny * P.nz;
  const size_t A = (size_t)P.nx * P.ny;
  double acc[6] = {0, 0, 0, 0, 0, 0};
  // node indices fit 32 bits (every population row stays below 4 GiB)
  const uint32_t nx = (uint32_t)P.nx, ny = (uint32_t)P.ny;
  for (uint32_t n = (uint32_t)(hs.k0 * A) + blockIdx.x * blockDim.x + threadIdx.x;
       n < (uint32_t)(hs.k1 * A); n += gridDim.x * blockDim.x) {
    const uint32_t r = n / nx;
    const int i = (int)(n - r * nx);
    const int j = (int)(r % ny);
    const int k = (int)(r / ny);
    R f[Q], g[Q];
    load_node<C>(in, N, (uint32_t)n, P, f, g);
    ScratchNb<R> nb{srho, sE, P, i, j, k, spsi};
    const Macro<R> m = macro_from_scratch<R>(f, g, nb, P);
    typename Codec<C>::T0 f0, g0;
    Codec<C>::ld0(in, (uint32_t)n, f0, g0);
    double rho = (double)f0, E = (double)g0;
#pragma unroll
    for (int l = 1; l < Q; ++l) {
      rho += (double)f[l];
      E += (double)g[l];
    }
    const double T = E / rho;
    const double vz = (double)m.vz;
    auto pick = [&](int q) {
      switch (q) {
        case LBM_Q_RHO: return rho;
        case LBM_Q_T: return T;
        case LBM_Q_VZ: return vz;
        default: return rho * (c_v * T + 0.25 * G * exp(-2.0 / rho)) * vz;   // rho U v_z
      }
    };
    const double x = pick(hs.qx);
    const double y = hs.qy >= 0 ? pick(hs.qy) : 0.0;
    acc[0] += 1.0;
    acc[1] += x;
    acc[2] += x * x;
    acc[3] += y;
    acc[4] += y * y;
    const double fx = (x - hs.xlo) * hs.xscale;
    const double fy = hs.qy >= 0 ? (y - hs.ylo) * hs.yscale : 0.0;
    if (fx >= 0.0 && fx < (double)hs.nxb && fy >= 0.0 && fy < (double)hs.nyb) {
      const int b = (int)fx * hs.nyb + (int)fy;
      if (lds)
        atomicAdd(&sh_bins[b], 1u);
      else
        atomicAdd(&counts[b], 1ull);
    } else {
      acc[5] += 1.0;
    }
  }
  __syncthreads();
  if (lds)
    for (int q = threadIdx.x; q < nbins; q += blockDim.x)
      if (sh_bins[q]) atomicAdd(&counts[q], (unsigned long long)sh_bins[q]);
  for (int q = 0; q < 6; ++q) {
    const double sum = block_sum(acc[q], sh);
    if (threadIdx.x == 0) partials[(size_t)blockIdx.x * 8 + q] = sum;
  }
}

// Numeric guard of lbm_step: per block, the FP64 sums of the stored mass
// and energy and the number of nodes whose stored populations sum to a
// non-finite value or to rho <= 0, into partials[blk * 8 + {0, 1, 2}].
template <typename C, typename R = typename C::R>
__global__ __launch_bounds__(256) void k_check(const typename C::S* __restrict__ in, DevParams<R> P,
                                               double* __restrict__ partials) {
  __shared__ double sh[4];
  const size_t N = (size_t)P.nx * P.ny * P.nz;
  double m = 0.0, e = 0.0, bad = 0.0;
  for (size_t n = blockIdx.x * (size_t)blockDim.x + threadIdx.x; n < N;
       n += (size_t)gridDim.x * blockDim.x) {
    typename Codec<C>::T0 f0, g0;
    Codec<C>::ld0(in, (uint32_t)n, f0, g0);
    double rho = (double)f0, E = (double)g0;
#pragma unroll
    for (int l = 1; l < Q; ++l) {
      R f, g;
      Codec<C>::dec(at32(Codec<C>::row(in, l, N), (uint32_t)n), f, g, P.fref[l], P.gref[l]);
      rho += (double)f;
      E += (double)g;
    }
    const bool b = !(rho > 0.0) || !isfinite(rho) || !isfinite(E);
    bad += b ? 1.0 : 0.0;
    m += b ? 0.0 : rho;
    e += b ? 0.0 : E;
  }
  const double sm = block_sum(m, sh);
  const double se = block_sum(e, sh);
  const double sb = block_sum(bad, sh);
  if (threadIdx.x == 0) {
    partials[(size_t)blockIdx.x * 8 + 0] = sm;
    partials[(size_t)blockIdx.x * 8 + 1] = se;
    partials[(size_t)blockIdx.x * 8 + 2] = sb;
    for (int q = 3; q < 7; ++q) partials[(size_t)blockIdx.x * 8 + q] = 0.0;
  }
}

__global__ void k_zero_u64(unsigned long long* p, size_t n) {
  for (size_t q = blockIdx.x * (size_t)blockDim.x + threadIdx.x; q < n;
       q += (size_t)gridDim.x * blockDim.x)
    p[q] = 0ull;
}

// Node quantity over planes [k0, k1) into q (FP64, node order within the
// planes), for the structure functions.
template <typename C, typename R = typename C::R>
__global__ __launch_bounds__(256) void k_quantity(const typename C::S* __restrict__ in,
                                                  const R* __restrict__ srho,
                                                  const R* __restrict__ sE,
                                                  const R* __restrict__ spsi, DevParams<R> P,
                                                  double c_v, double G, int k0, int k1, int which,
                                                  double* __restrict__ q) {
  const size_t N = (size_t)P.nx * P.ny * P.nz;
  const size_t A = (size_t)P.nx * P.ny;
  for (size_t n = (size_t)k0 * A + blockIdx.x * (size_t)blockDim.x + threadIdx.x;
       n < (size_t)k1 * A; n += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(n % P.nx);
    const int j = (int)((n / P.nx) % P.ny);
    const int k = (int)(n / A);
    R f[Q], g[Q];
    load_node<C>(in, N, (uint32_t)n, P, f, g);
    ScratchNb<R> nb{srho, sE, P, i, j, k, spsi};
    const Macro<R> m = macro_from_scratch<R>(f, g, nb, P);
    typename Codec<C>::T0 f0, g0;
    Codec<C>::ld0(in, (uint32_t)n, f0, g0);
    double rho = (double)f0, E = (double)g0;
#pragma unroll
    for (int l = 1; l < Q; ++l) {
      rho += (double)f[l];
      E += (double)g[l];
    }
    const double T = E / rho;
    double v;
    switch (which) {
      case LBM_Q_RHO: v = rho; break;
      case LBM_Q_T: v = T; break;
      case LBM_Q_VZ: v = (double)m.vz; break;
      default: v = rho * (c_v * T + 0.25 * G * exp(-2.0 / rho)) * (double)m.vz; break;
    }
    q[n - (size_t)k0 * A] = v;
  }
}

// Horizontal increments of a field a (planes of nx x ny, `planes` of them):
// every work-group takes whole lines (along x for line < planes*ny, along y
// after that) into LDS; thread t handles separation r = t + 1 and sums
// (a(x + r e) - a(x))^2 and ^4 over the line (periodic).  Per-block partials
// [block][r][2] go to `part`.
__global__ __launch_bounds__(256) void k_increments(const double* __restrict__ a, int nx, int ny,
                                                    int planes, int rmax,
                                                    double* __restrict__ part) {
  extern __shared__ double line[];
  const int t = threadIdx.x;
  const long long nlx = (long long)planes * ny, nly = (long long)planes * nx;
  double s2 = 0.0, s4 = 0.0;
  for (long long L = blockIdx.x; L < nlx + nly; L += gridDim.x) {
    int len;
    __syncthreads();
    if (L < nlx) {  // line along x: plane p, row j
      len = nx;
      const double* src = a + (size_t)L * nx;
      for (int q = t; q < nx; q += blockDim.x) line[q] = src[q];
    } else {        // line along y: plane p, column i
      len = ny;
      const long long c = L - nlx;
      const int p = (int)(c / nx), i = (int)(c % nx);
      const double* src = a + (size_t)p * nx * ny + i;
      for (int q = t; q < ny; q += blockDim.x) line[q] = src[(size_t)q * nx];
    }
    __syncthreads();
    const int r = t + 1;
    if (r <= rmax && r < len) {
      for (int q = 0; q < len; ++q) {
        const int qr = q + r < len ? q + r : q + r - len;
        const double d = line[qr] - line[q];
        const double d2 = d * d;
        s2 += d2;
        s4 += d2 * d2;
      }
    }
  }
  if (t < rmax) {
    part[((size_t)blockIdx.x * rmax + t) * 2] = s2;
    part[((size_t)blockIdx.x * rmax + t) * 2 + 1] = s4;
  }
}

// out[r][2] = sum over blocks of part[block][r][2], fixed order.
__global__ void k_finish_increments(const double* __restrict__ part, int nblk, int rmax,
                                    double* __restrict__ out) {
  for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < rmax; r += gridDim.x * blockDim.x) {
    double s2 = 0.0, s4 = 0.0;
    for (int b = 0; b < nblk; ++b) {
      s2 += part[((size_t)b * rmax + r) * 2];
      s4 += part[((size_t)b * rmax + r) * 2 + 1];
    }
    out[2 * r] = s2;
    out[2 * r + 1] = s4;
  }
}

// Fixed-order sum of the block partials (deterministic).
__global__ __launch_bounds__(256) void k_finish_totals(const double* __restrict__ partials,
                                                       int nblk, double* __restrict__ out) {
  __shared__ double sh[4];
  for (int q = 0; q < 7; ++q) {
    double v = 0.0;
    for (int b = threadIdx.x; b < nblk; b += blockDim.x) v += partials[(size_t)b * 8 + q];
    const double s = block_sum(v, sh);
    if (threadIdx.x == 0) out[q] = s;
  }
}

// Horizontal averages per plane: prof[2k] = mean T, prof[2k+1] = mean rho U v_z.
template <typename C, typename R = typename C::R>
__global__ __launch_bounds__(256) void k_plane(const typename C::S* __restrict__ in,
                                               const R* __restrict__ srho, const R* __restrict__ sE,
                                               const R* __restrict__ spsi,
                                               DevParams<R> P, double c_v, double G, int S,
                                               double* __restrict__ out) {
  __shared__ double sh[4];
  // S blocks per plane: block b = k S + s sums nodes s blockDim + t, stepping
  // S blockDim; with S = 1 it writes the plane's averages to out[2 k], else
  // its two sums to out[2 b] (k_plane_sum adds the slices in order)
  const int k = blockIdx.x / S, sl = blockIdx.x - k * S;
  const size_t N = (size_t)P.nx * P.ny * P.nz;
  const int plane = P.nx * P.ny;
  double sT = 0.0, sF = 0.0;
  for (int q = sl * blockDim.x + threadIdx.x; q < plane; q += S * blockDim.x) {
    const int i = q % P.nx, j = q / P.nx;
    const uint32_t n = node_off(i, j, k, P.nx, P.ny);
    R f[Q], g[Q];
    load_node<C>(in, N, (uint32_t)n, P, f, g);
    ScratchNb<R> nb{srho, sE, P, i, j, k, spsi};
    const Macro<R> m = macro_from_scratch<R>(f, g, nb, P);
    const double rho = m.rho, T = m.T;
    const double U = c_v * T + 0.25 * G * exp(-2.0 / rho);
    sT += T;
    sF += rho * U * (double)m.vz;
  }
  const double a = block_sum(sT, sh);
  const double b = block_sum(sF, sh);
  if (threadIdx.x == 0) {
    if (S == 1) {
      out[2 * k] = a / plane;
      out[2 * k + 1] = b / plane;
    } else {
      out[2 * blockIdx.x] = a;
      out[2 * blockIdx.x + 1] = b;
    }
  }
}

// plane averages from the S slice sums of each plane, added in slice order
__global__ void k_plane_sum(const double* __restrict__ part, int S, int nz, int plane,
                            double* __restrict__ prof) {
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < nz; k += gridDim.x * blockDim.x) {
    double a = 0.0, b = 0.0;
    for (int sl = 0; sl < S; ++sl) {
      a += part[2 * (k * S + sl)];
      b += part[2 * (k * S + sl) + 1];
    }
    prof[2 * k] = a / plane;
    prof[2 * k + 1] = b / plane;
  }
}

// <P d_j v_j>(k) from the moment fields (rho, vx, vy, vz, T): P = rho T +
// (G/2) psi^2 (the bulk equation of state), the divergence of the physical
// velocity on the W stencil with the ghost planes of the walls holding the
// negative mirror image (v = 0 on the half-way wall), periodic otherwise.
// One block per plane, FP64, fixed summation order.
__global__ __launch_bounds__(256) void k_pwork(const double* __restrict__ fl, int nx, int ny,
                                               int nz, int periodic, double G, int psi_form,
                                               double* __restrict__ prof) {
  __shared__ double sh[4];
  const int k = blockIdx.x;
  const size_t N = (size_t)nx * ny * nz;
  const int plane = nx * ny;
  double acc = 0.0;
  for (int q = threadIdx.x; q < plane; q += blockDim.x) {
    const int i = q % nx, j = q / nx;
    const size_t n = ((size_t)k * ny + j) * nx + i;
    const double rho = fl[n], T = fl[4 * N + n];
    const double psi = psi_form ? 1.0 - exp(-rho) : exp(-1.0 / rho);
    const double Pn = rho * T + 0.5 * G * psi * psi;
    double div = 0.0;
#pragma unroll
    for (int l = 1; l < Q; ++l) {
      const int ii = wrap(i + CX[l], nx), jj = wrap(j + CY[l], ny);
      int kk = k + CZ[l];
      double sgn = 1.0;
      if (kk < 0 || kk >= nz) {
        if (periodic) {
          kk = kk < 0 ? kk + nz : kk - nz;
        } else {
          kk = kk < 0 ? 0 : nz - 1;
          sgn = -1.0;
        }
      }
      const size_t m = ((size_t)kk * ny + jj) * nx + ii;
      const double cv = (double)CX[l] * fl[N + m] + (double)CY[l] * fl[2 * N + m] +
                        (double)CZ[l] * fl[3 * N + m];
      div += (l < 7 ? 1.0 / 6.0 : 1.0 / 12.0) * sgn * cv;
    }
    acc += Pn * div;
  }
  const double sum = block_sum(acc, sh);
  if (threadIdx.x == 0) prof[k] = sum / plane;
}

// Nusselt numbers from the plane profiles; out = [nu_bot, nu_top, nu_z[nz], T_z[nz]].
__global__ void k_finish_nusselt(const double* __restrict__ prof, int nz, double T_d, double T_u,
                                 double kappa, double* __restrict__ out) {
  const double dT = T_d - T_u;
  for (int k = threadIdx.x; k < nz; k += blockDim.x) {
    const double Tk = prof[2 * k];
    const double Tm = k > 0 ? prof[2 * (k - 1)] : 2.0 * T_d - prof[0];
    const double Tp = k < nz - 1 ? prof[2 * (k + 1)] : 2.0 * T_u - prof[2 * (nz - 1)];
    out[2 + k] = (prof[2 * k + 1] - kappa * 0.5 * (Tp - Tm)) * nz / (kappa * dT);
    out[2 + nz + k] = Tk;
  }
  if (threadIdx.x == 0) {
    out[0] = 2.0 * nz * (T_d - prof[0]) / dT;
    out[1] = 2.0 * nz * (prof[2 * (nz - 1)] - T_u) / dT;
  }
}

// ---------------------------------------------------------------- adjoint
//
// Discrete adjoint of one step (the transpose of its Jacobian applied to
// lambda_{t+1} = dJ/d state_{t+1}), in the handle's compute precision.  The
// forward state is given in canonical FP64 form.  Three passes:
//   k_adj_rhoE     rho and E of the forward state (for the stencils),
//   k_adj_local    adjoint of streaming (gather) and of the node-local
//                  collision, leaving the adjoints of the three stencil
//                  gradients per node in scratch,
//   k_adj_stencil  transpose of the gradient stencils (with the wall ghosts)
//                  added to lambda_t.

template <typename R>
__global__ void k_adj_rhoE(const double* __restrict__ st, R* __restrict__ srho,
                           R* __restrict__ sE, DevParams<R> P) {
  const size_t N = (size_t)P.nx * P.ny * P.nz;
  for (size_t n = blockIdx.x * (size_t)blockDim.x + threadIdx.x; n < N;
       n += (size_t)gridDim.x * blockDim.x) {
    R r = R(0), e = R(0);
#pragma unroll
    for (int l = 0; l < Q; ++l) {
      r += (R)st[(size_t)l * N + n];
      e += (R)st[(size_t)(l + Q) * N + n];
    }
    srho[n] = r;
    sE[n] = e;
  }
}

template <typename R>
__global__ __launch_bounds__(256) void k_adj_local(const double* __restrict__ st,
                                                   const double* __restrict__ lam1,
                                                   double* __restrict__ lam0,
                                                   const R* __restrict__ srho,
                                                   const R* __restrict__ sE, R* __restrict__ gbar,
                                                   DevParams<R> P, double* __restrict__ partials) {
  __shared__ double sh[4];
  const size_t N = (size_t)P.nx * P.ny * P.nz;
  double accG = 0.0, accTd = 0.0;
  for (size_t n = blockIdx.x * (size_t)blockDim.x + threadIdx.x; n < N;
       n += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(n % P.nx);
    const int j = (int)((n / P.nx) % P.ny);
    const int k = (int)(n / ((size_t)P.nx * P.ny));
    // forward quantities
    R f[Q], g[Q];
#pragma unroll
    for (int l = 0; l < Q; ++l) {
      f[l] = (R)st[(size_t)l * N + n];
      g[l] = (R)st[(size_t)(l + Q) * N + n];
    }
    R rho, E;
    moments<R>(f, g, rho, E);
    ScratchNb<R> nb{srho, sE, P, i, j, k};
    R gpx, gpy, gpz, gEx, gEy, gEz, grx, gry, grz;
    grad_w<R>([&](int l) { return nb.get(0, l); }, gpx, gpy, gpz);
    grad_w<R>([&](int l) { return nb.get(2, l); }, gEx, gEy, gEz);
    grad_w<R>([&](int l) { return nb.get(1, l); }, grx, gry, grz);
    const R psi = psi_of<R>(rho, P.psi_form);
    const Macro<R> m = node_macro<R>(f, g, rho, E, psi, gpx, gpy, gpz, gEx, gEy, gEz, grx, gry,
                                     grz, P);
    const R ir = R(1) / rho;
    const R ux = (m.jx + P.tau_nu * m.Fx) * ir;
    const R uy = (m.jy + P.tau_nu * m.Fy) * ir;
    const R uz = (m.jz + P.tau_nu * m.Fz) * ir;
    const R uu = R(1) - R(1.5) * (ux * ux + uy * uy + uz * uz);
    const R vv = R(-1.5) * (m.vx * m.vx + m.vy * m.vy + m.vz * m.vz);

    // adjoint of streaming: lambda of the collided populations
    R as[Q], bs[Q];
#pragma unroll
    for (int l = 0; l < Q; ++l) {
      int kk = k + CZ[l];
      const int ii = wrap(i + CX[l], P.nx), jj = wrap(j + CY[l], P.ny);
      if (kk >= 0 && kk < P.nz) {
        const size_t o = ((size_t)kk * P.ny + jj) * P.nx + ii;
        as[l] = (R)lam1[(size_t)l * N + o];
        bs[l] = (R)lam1[(size_t)(l + Q) * N + o];
      } else if (P.periodic_z) {
        kk = kk < 0 ? kk + P.nz : kk - P.nz;
        const size_t o = ((size_t)kk * P.ny + jj) * P.nx + ii;
        as[l] = (R)lam1[(size_t)l * N + o];
        bs[l] = (R)lam1[(size_t)(l + Q) * N + o];
      } else {
        const double lg = lam1[(size_t)(OPP[l] + Q) * N + n];
        as[l] = (R)lam1[(size_t)OPP[l] * N + n];
        bs[l] = (R)(-lg);
        if (kk < 0) accTd += 2.0 * wlat<double>(l) * (double)P.rho_kappa * lg;
      }
    }

    // adjoint of the BGK collisions
    R rb = R(0), Eb = R(0), sbar = R(0);
    R ubx = R(0), uby = R(0), ubz = R(0), vbx = R(0), vby = R(0), vbz = R(0);
    const R gE = P.gamma * m.E;
#pragma unroll
    for (int l = 0; l < Q; ++l) {
      const R w = wlat<R>(l);
      const R cx = R(CX[l]), cy = R(CY[l]), cz = R(CZ[l]);
      const R A = P.omega_f * as[l];
      const R cu = cx * ux + cy * uy + cz * uz;
      const R feq_over_rho = w * (uu + cu * (R(3) + R(4.5) * cu)) + af<R>(l) * (P.T_lat - R(1) / R(3));
      rb += A * feq_over_rho;
      const R cf = A * w * rho;
      const R tf = R(3) + R(9) * cu;
      ubx += cf * (tf * cx - R(3) * ux);
      uby += cf * (tf * cy - R(3) * uy);
      ubz += cf * (tf * cz - R(3) * uz);
      const R B = P.omega_g * bs[l];
      sbar += w * bs[l];
      const R cv = cx * m.vx + cy * m.vy + cz * m.vz;
      Eb += B * (w * (R(1) + P.gamma * (vv + cv * (R(3) + R(4.5) * cv))) +
                 bg<R>(l) * (P.rho_kappa * ir - R(1)));
      rb += B * bg<R>(l) * (-P.rho_kappa * m.E * ir * ir);
      const R cg = B * w * gE;
      const R tg = R(3) + R(9) * cv;
      vbx += cg * (tg * cx - R(3) * m.vx);
      vby += cg * (tg * cy - R(3) * m.vy);
      vbz += cg * (tg * cz - R(3) * m.vz);
    }
    // counter-term source S = (v . grad E) / c_v
    vbx += sbar * gEx * P.inv_cv;
    vby += sbar * gEy * P.inv_cv;
    vbz += sbar * gEz * P.inv_cv;
    R GEbx = sbar * m.vx * P.inv_cv, GEby = sbar * m.vy * P.inv_cv, GEbz = sbar * m.vz * P.inv_cv;
    // u' = (j + tau F)/rho and v = (j + F/2)/rho
    const R jbx = (ubx + vbx) * ir, jby = (uby + vby) * ir, jbz = (ubz + vbz) * ir;
    const R Fbx = (P.tau_nu * ubx + R(0.5) * vbx) * ir;
    const R Fby = (P.tau_nu * uby + R(0.5) * vby) * ir;
    const R Fbz = (P.tau_nu * ubz + R(0.5) * vbz) * ir;
    rb -= (ubx * ux + uby * uy + ubz * uz + vbx * m.vx + vby * m.vy + vbz * m.vz) * ir;
    // F = -G psi grad psi - (grad E - T_lat grad rho) - g rho z
    const R Fdotgp = Fbx * gpx + Fby * gpy + Fbz * gpz;
    const R psib = -P.G * Fdotgp;
    accG += -(double)psi * (double)Fdotgp;
    const R Gpbx = -P.G * psi * Fbx, Gpby = -P.G * psi * Fby, Gpbz = -P.G * psi * Fbz;
    GEbx -= Fbx;
    GEby -= Fby;
    GEbz -= Fbz;
    const R Grbx = P.T_lat * Fbx, Grby = P.T_lat * Fby, Grbz = P.T_lat * Fbz;
    rb -= P.gravity * Fbz;
    rb += P.psi_form ? psib * (R(1) - psi) : psib * psi * ir * ir;   // d psi / d rho

#pragma unroll
    for (int l = 0; l < Q; ++l) {
      lam0[(size_t)l * N + n] = (double)((R(1) - P.omega_f) * as[l] + rb +
                                         (R(CX[l]) * jbx + R(CY[l]) * jby + R(CZ[l]) * jbz));
      lam0[(size_t)(l + Q) * N + n] = (double)((R(1) - P.omega_g) * bs[l] + Eb);
    }
    gbar[n] = Gpbx;
    gbar[N + n] = Gpby;
    gbar[2 * N + n] = Gpbz;
    gbar[3 * N + n] = GEbx;
    gbar[4 * N + n] = GEby;
    gbar[5 * N + n] = GEbz;
    gbar[6 * N + n] = Grbx;
    gbar[7 * N + n] = Grby;
    gbar[8 * N + n] = Grbz;
  }
  const double sG = block_sum(accG, sh);
  const double sT = block_sum(accTd, sh);
  if (threadIdx.x == 0) {
    partials[(size_t)blockIdx.x * 8] = sG;
    partials[(size_t)blockIdx.x * 8 + 1] = sT;
  }
}

template <typename R>
__device__ __forceinline__ R wdot(const R* gbar, size_t N, int comp, size_t o, int l) {
  return R(CX[l]) * gbar[(size_t)(3 * comp) * N + o] + R(CY[l]) * gbar[(size_t)(3 * comp + 1) * N + o] +
         R(CZ[l]) * gbar[(size_t)(3 * comp + 2) * N + o];
}

template <typename R>
__global__ __launch_bounds__(256) void k_adj_stencil(const R* __restrict__ srho,
                                                     const R* __restrict__ gbar,
                                                     double* __restrict__ lam0, DevParams<R> P) {
  const size_t N = (size_t)P.nx * P.ny * P.nz;
  for (size_t n = blockIdx.x * (size_t)blockDim.x + threadIdx.x; n < N;
       n += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(n % P.nx);
    const int j = (int)((n / P.nx) % P.ny);
    const int k = (int)(n / ((size_t)P.nx * P.ny));
    R pb = R(0), eb = R(0), qb = R(0);   // adjoints of psi, E, rho at this node
#pragma unroll
    for (int l = 1; l < Q; ++l) {
      const R W = l < 7 ? R(1) / R(6) : R(1) / R(12);
      const int ix = wrap(i - CX[l], P.nx), jx = wrap(j - CY[l], P.ny);
      int kx = k - CZ[l];
      bool real = kx >= 0 && kx < P.nz;
      if (!real && P.periodic_z) {
        kx = kx < 0 ? kx + P.nz : kx - P.nz;
        real = true;
      }
      if (real) {  // node x = y - c_l reads this node in direction l
        const size_t o = ((size_t)kx * P.ny + jx) * P.nx + ix;
        pb += W * wdot(gbar, N, 0, o, l);
        eb += W * wdot(gbar, N, 1, o, l);
        qb += W * wdot(gbar, N, 2, o, l);
      }
      if (!P.periodic_z) {
        // ghosts: a node x on a wall plane reading direction l across the
        // wall sees psi of the wall-plane node (mirror; a constant, with no
        // adjoint, for a prescribed wall density) and 2 a(wall plane)
        // - a(next plane) for E and rho (linear extrapolation)
        const int kw = CZ[l] < 0 ? 0 : P.nz - 1;
        const int ki = CZ[l] < 0 ? 1 : P.nz - 2;
        const int wet = CZ[l] < 0 ? P.wet_d : P.wet_u;
        if (CZ[l] != 0 && (k == kw || k == ki)) {
          const size_t o = ((size_t)kw * P.ny + jx) * P.nx + ix;
          if (k == kw) {
            if (!wet) pb += W * wdot(gbar, N, 0, o, l);
            eb += R(2) * W * wdot(gbar, N, 1, o, l);
            qb += R(2) * W * wdot(gbar, N, 2, o, l);
          }
          if (k == ki) {
            eb -= W * wdot(gbar, N, 1, o, l);
            qb -= W * wdot(gbar, N, 2, o, l);
          }
        }
      }
    }
    const R rho = srho[n];
    const R psi = psi_of<R>(rho, P.psi_form);
    const double addf = (double)(qb + (P.psi_form ? pb * (R(1) - psi) : pb * psi / (rho * rho)));
    const double addg = (double)eb;
#pragma unroll
    for (int l = 0; l < Q; ++l) {
      lam0[(size_t)l * N + n] += addf;
      lam0[(size_t)(l + Q) * N + n] += addg;
    }
  }
}

// lambda += weight * d q_bot / d state, q_bot = 2 kappa (T_d - mean_{k=0} E/rho);
// out[blockIdx] partial of sum_{k=0} E/rho.
template <typename R>
__global__ __launch_bounds__(256) void k_adj_qbot(const double* __restrict__ st,
                                                  double* __restrict__ lam, DevParams<R> P,
                                                  double weight, double kappa,
                                                  double* __restrict__ partials) {
  __shared__ double sh[4];
  const size_t N = (size_t)P.nx * P.ny * P.nz;
  const size_t A = (size_t)P.nx * P.ny;
  double accT = 0.0;
  for (size_t n = blockIdx.x * (size_t)blockDim.x + threadIdx.x; n < A;
       n += (size_t)gridDim.x * blockDim.x) {
    double rho = 0.0, E = 0.0;
    for (int l = 0; l < Q; ++l) {
      rho += st[(size_t)l * N + n];
      E += st[(size_t)(l + Q) * N + n];
    }
    accT += E / rho;
    const double df = weight * 2.0 * kappa * E / (rho * rho * (double)A);
    const double dg = -weight * 2.0 * kappa / (rho * (double)A);
    if (lam) {
      for (int l = 0; l < Q; ++l) {
        lam[(size_t)l * N + n] += df;
        lam[(size_t)(l + Q) * N + n] += dg;
      }
    }
  }
  const double s = block_sum(accT, sh);
  if (threadIdx.x == 0) partials[(size_t)blockIdx.x * 8] = s;
}

// dJ/drho0 from lambda_0: f = w rho0 + a rho0 (T_lat - 1/3),
// g = w rho0 T0 + b (rho_kappa - rho0) T0.
template <typename R>
__global__ void k_adj_init(const double* __restrict__ lam, const double* __restrict__ T0,
                           double* __restrict__ out, DevParams<R> P) {
  const size_t N = (size_t)P.nx * P.ny * P.nz;
  for (size_t n = blockIdx.x * (size_t)blockDim.x + threadIdx.x; n < N;
       n += (size_t)gridDim.x * blockDim.x) {
    const int k = (int)(n / ((size_t)P.nx * P.ny));
    const double T = T0 ? T0[n]
                        : (double)P.T_d + ((double)P.T_u - (double)P.T_d) * ((double)k + 0.5) / (double)P.nz;
    double s = 0.0;
    for (int l = 0; l < Q; ++l)
      s += (wlat<double>(l) + af<double>(l) * ((double)P.T_lat - 1.0 / 3.0)) * lam[(size_t)l * N + n] +
           (wlat<double>(l) - bg<double>(l)) * T * lam[(size_t)(l + Q) * N + n];
    out[n] = s;
  }
}

// ---------------------------------------------------------------- host side

constexpr size_t kAlign = 256;
size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// bytes of one stored population (a stored word holds the pair f_l, g_l)
// Bytes of one node's populations in one buffer, and of the widest row (one
// direction's array), which must stay below 4 GiB for the 32-bit offsets.
size_t node_bytes(int storage) {
  switch (storage) {
    case LBM_FP64: return Q * 16;
    case LBM_FP32: return Q * 8;
    default: return (Q - 1) * 4 + 8;   // 18 moving 16-bit pairs + the FP32 rest pair
  }
}
size_t row_bytes(int storage) { return storage == LBM_FP64 ? 16 : 8; }
size_t real_bytes(int storage) { return storage == LBM_FP64 ? 8 : 4; }

constexpr int kDiagBlocks = 1024;

int validate(const lbm_params* p) {
  if (!p) return fail(LBM_EINVAL, "params is NULL");
  if (p->nx < 1 || p->ny < 1 || p->nz < 1) return fail(LBM_EINVAL, "nx, ny, nz must be >= 1");
  if (!p->periodic_z && p->nz < 2) return fail(LBM_EINVAL, "walls need nz >= 2");
  if ((double)p->nx * p->ny * p->nz * (double)row_bytes(p->storage) >= 4294967296.0)
    return fail(LBM_EINVAL, "lattice too large (one direction's population array must stay below 4 GiB)");
  if (p->storage < LBM_FP64 || p->storage > LBM_BF16DEV) return fail(LBM_EINVAL, "unknown storage");
  if (p->kernel != LBM_KERNEL_FUSED && p->kernel != LBM_KERNEL_REFERENCE &&
      p->kernel != LBM_KERNEL_FUSED_RELOAD && p->kernel != LBM_KERNEL_PIPELINED)
    return fail(LBM_EINVAL, "unknown kernel");
  if (p->kernel == LBM_KERNEL_PIPELINED) {
    if (p->storage == LBM_FP64)
      return fail(LBM_EINVAL, "the pipelined kernel is built for FP32 and the 16-bit forms only");
    const int tx = p->tile_x, ty = p->tile_y;
    const bool ok = (tx == 0 && ty == 0) || (tx == 32 && (ty == 8 || ty == 16)) ||
                    (tx == 64 && ty == 8) || (tx == 16 && ty == 16) || (tx == 128 && ty == 4) ||
                    (tx == 256 && ty == 2);
    if (!ok) return fail(LBM_EINVAL, "unsupported tile shape (tile_x, tile_y) for the pipelined kernel");
  } else {
    const int tx = p->tile_x, ty = p->tile_y;
    const bool ok = (tx == 0 && ty == 0) ||
                    (tx == 64 && (ty == 1 || ty == 2 || ty == 4 || ty == 8 || ty == 16)) ||
                    (tx == 32 && (ty == 8 || ty == 16 || ty == 32)) ||
                    (tx == 0 && (ty == 1 || ty == 2 || ty == 4 || ty == 8 || ty == 16));
    if (!ok) return fail(LBM_EINVAL, "unsupported tile shape (tile_x, tile_y)");
  }
  if (p->z_chunk < 0) return fail(LBM_EINVAL, "z_chunk must be >= 0");
  if (!(p->tau_nu > 0.5) || !(p->tau_kappa > 0.5)) return fail(LBM_EINVAL, "tau must be > 1/2");
  if (!(p->G <= 0.0) || !isfinite(p->G)) return fail(LBM_EINVAL, "G must be <= 0 and finite");
  if (!(p->c_v > 0.0) || !(p->rho_kappa > 0.0)) return fail(LBM_EINVAL, "c_v and rho_kappa must be > 0");
  if (!(p->T_d > 0.0) || !(p->T_u > 0.0)) return fail(LBM_EINVAL, "wall temperatures must be > 0");
  if (!isfinite(p->gravity)) return fail(LBM_EINVAL, "gravity must be finite");
  if (!isfinite(p->rho_wall_d) || !isfinite(p->rho_wall_u))
    return fail(LBM_EINVAL, "wall densities must be finite");
  if (p->psi_form != 0 && p->psi_form != 1) return fail(LBM_EINVAL, "psi_form must be 0 or 1");
  if (p->storage >= LBM_FP16DEV && (!(p->rho_ref > 0.0) || !(p->T_ref > 0.0)))
    return fail(LBM_EINVAL, "16-bit storage needs rho_ref > 0 and T_ref > 0");
  return LBM_OK;
}

struct Layout {
  size_t N, pop_bytes, buf, scr, part, small, adj, total;
};

Layout layout(const lbm_params* p) {
  Layout L;
  L.N = (size_t)p->nx * p->ny * p->nz;
  // node_bytes = the words of one node in all its rows; rows are row_pitch(N) apart
  L.pop_bytes = align_up(row_pitch(L.N) * node_bytes(p->storage));
  L.buf = L.pop_bytes;
  L.scr = align_up(L.N * real_bytes(p->storage));
  L.part = align_up((size_t)kDiagBlocks * 8 * sizeof(double));
  L.small = align_up((size_t)(16 + 4 * p->nz) * sizeof(double));
  // adjoint scratch, FP64 for every storage form: 9 gradient-adjoint
  // components plus rho and E of the forward state
  L.adj = p->adjoint ? align_up((size_t)11 * L.N * sizeof(double)) : 0;
  L.total = 2 * L.buf + 3 * L.scr + L.part + 2 * L.small + L.adj;
  return L;
}

}  // namespace

struct lbm_handle {
  lbm_params p;
  Layout L;
  int dev;         // the HIP device current at lbm_init
  hipStream_t stream;
  char* ws;
  void* buf[2];
  void* srho;
  void* sE;
  void* spsi;      // psi of the state in srho (written with it)
  double* partials;
  double* small;   // totals / nusselt results
  double* prof;    // plane profiles (2 nz)
  double* gbar;    // adjoint scratch (9 N doubles) or NULL
  double* arho;    // rho and E of the state the adjoint step linearises about
  double* aE;
  int cur;
  int64_t t;
  int64_t state_version;  // bumped whenever buf[cur] changes (init, step, set_state)
  int64_t rhoE_version;   // the state version srho / sE were computed for
  int kernel, tile_x, tile_y, z_chunk;
  int64_t check_every;   // numeric guard interval of lbm_step (0 = off)
  double check_mass_tol; // relative mass change that counts as a failure
  double check_mass0;    // stored mass at the first check after init / set_state (0 = not yet)
};

namespace {

template <typename R>
DevParams<R> dev_params(const lbm_params& p) {
  DevParams<R> d;
  d.nx = p.nx;
  d.ny = p.ny;
  d.nz = p.nz;
  d.periodic_z = p.periodic_z ? 1 : 0;
  d.omega_f = (R)(1.0 / p.tau_nu);
  d.omega_g = (R)(1.0 / p.tau_kappa);
  d.tau_nu = (R)p.tau_nu;
  d.G = (R)p.G;
  d.gravity = (R)p.gravity;
  d.inv_cv = (R)(1.0 / p.c_v);
  d.gamma = (R)(1.0 + 1.0 / p.c_v);
  d.rho_kappa = (R)p.rho_kappa;
  d.T_d = (R)p.T_d;
  d.T_u = (R)p.T_u;
  const double T_lat = p.T_lat > 0.0 ? p.T_lat : 0.5 * (p.T_d + p.T_u);
  d.T_lat = (R)T_lat;
  d.wet_d = p.rho_wall_d > 0.0 ? 1 : 0;
  d.wet_u = p.rho_wall_u > 0.0 ? 1 : 0;
  d.psi_form = p.psi_form;
  auto psi_host = [&](double r) { return p.psi_form ? 1.0 - exp(-r) : exp(-1.0 / r); };
  d.psi_wd = (R)(d.wet_d ? psi_host(p.rho_wall_d) : 0.0);
  d.psi_wu = (R)(d.wet_u ? psi_host(p.rho_wall_u) : 0.0);
  const bool dev = p.storage >= LBM_FP16DEV;
  for (int l = 0; l < Q; ++l) {
    // reference populations: equilibrium at rest of (rho_ref, T_ref)
    const double E = p.rho_ref * p.T_ref;
    const double w = wlat<double>(l);
    d.fref[l] = dev ? (R)(w * p.rho_ref + af<double>(l) * p.rho_ref * (T_lat - 1.0 / 3.0)) : R(0);
    d.gref[l] = dev ? (R)(w * E + bg<double>(l) * (p.rho_kappa - p.rho_ref) * p.T_ref) : R(0);
  }
  return d;
}

int grid_for(size_t n, int block) {
  size_t g = (n + block - 1) / block;
  if (g > 65536) g = 65536;
  if (g < 1) g = 1;
  return (int)g;
}

template <typename C, int TX, int TY, bool KEEP>
int launch_tile(lbm_handle* h, const void* in, void* out) {
  using R = typename C::R;
  const DevParams<R> P = dev_params<R>(h->p);
  const int ntx = (h->p.nx + TX - 1) / TX, nty = (h->p.ny + TY - 1) / TY;
  const int kz = h->z_chunk;
  const int nzc = (h->p.nz + kz - 1) / kz;
  const long long nblk = (long long)ntx * nty * nzc;
  if (nblk > 0x7fffffffLL) return fail(LBM_EINVAL, "grid too large");
  hipLaunchKernelGGL((k_fused<C, TX, TY, KEEP>), dim3((unsigned)nblk), dim3(TX * TY), 0, h->stream,
                     (const typename C::S*)in, (typename C::S*)out, P, ntx, nty, kz);
  HIP_TRY(hipGetLastError());
  return LBM_OK;
}

// Tile shapes (TX x TY) the library is built for: f(TX, TY, KEEP) is called
// with the shape as integral constants.  Keeping the next plane in registers
// is only built for tiles of at most 512 threads.
template <bool KEEP, typename F>
int with_tile(int tx, int ty, F&& f) {
  using std::bool_constant;
  using std::integral_constant;
  using I64 = integral_constant<int, 64>;
  using I32 = integral_constant<int, 32>;
  if (tx == 64) {
    switch (ty) {
      case 1: return f(I64{}, integral_constant<int, 1>{}, bool_constant<KEEP>{});
      case 2: return f(I64{}, integral_constant<int, 2>{}, bool_constant<KEEP>{});
      case 4: return f(I64{}, integral_constant<int, 4>{}, bool_constant<KEEP>{});
      case 8: return f(I64{}, integral_constant<int, 8>{}, bool_constant<KEEP>{});
      case 16: return f(I64{}, integral_constant<int, 16>{}, bool_constant<false>{});
    }
  } else if (tx == 32) {
    switch (ty) {
      case 8: return f(I32{}, integral_constant<int, 8>{}, bool_constant<KEEP>{});
      case 16: return f(I32{}, integral_constant<int, 16>{}, bool_constant<KEEP>{});
      case 32: return f(I32{}, integral_constant<int, 32>{}, bool_constant<false>{});
    }
  }
  return fail(LBM_EINVAL, "unsupported tile shape");
}

template <typename C, bool KEEP>
int launch_fused(lbm_handle* h, const void* in, void* out) {
  return with_tile<KEEP>(h->tile_x, h->tile_y, [&](auto X, auto Y, auto K) {
    return launch_tile<C, decltype(X)::value, decltype(Y)::value, decltype(K)::value>(h, in, out);
  });
}

// Work-groups of the fused kernel for this tile that one compute unit holds
// at once (registers and LDS decide), or <= 0 if the runtime cannot tell.
template <typename C, bool KEEP>
int fused_groups_per_cu(int tx, int ty) {
  return with_tile<KEEP>(tx, ty, [&](auto X, auto Y, auto K) {
    constexpr int TX = decltype(X)::value, TY = decltype(Y)::value;
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_fused<C, TX, TY, decltype(K)::value>,
                                                     TX * TY, 0) != hipSuccess)
      return 0;
    return nb;
  });
}

pipe::PParams pipe_params(const lbm_params& p) {
  pipe::PParams d;
  d.nx = p.nx;
  d.ny = p.ny;
  d.nz = p.nz;
  d.periodic_z = p.periodic_z ? 1 : 0;
  d.omega_f = (float)(1.0 / p.tau_nu);
  d.omega_g = (float)(1.0 / p.tau_kappa);
  d.tau_nu = (float)p.tau_nu;
  d.G = (float)p.G;
  d.gravity = (float)p.gravity;
  d.inv_cv = (float)(1.0 / p.c_v);
  d.gamma = (float)(1.0 + 1.0 / p.c_v);
  d.rho_kappa = (float)p.rho_kappa;
  d.T_d = (float)p.T_d;
  d.T_u = (float)p.T_u;
  const double T_lat = p.T_lat > 0.0 ? p.T_lat : 0.5 * (p.T_d + p.T_u);
  d.T_lat = (float)T_lat;
  const bool dev = p.storage >= LBM_FP16DEV;
  d.rho_ref0 = dev ? (float)p.rho_ref : 0.f;
  d.T_ref0 = dev ? (float)p.T_ref : 0.f;
  // sums of the FP32 reference populations of the moving directions (the
  // values the 16-bit words are deviations from; the same as dev_params)
  double sf = 0.0, sg = 0.0;
  for (int l = 1; l < Q; ++l) {
    const double w = wlat<double>(l);
    sf += (double)(float)(w * p.rho_ref + af<double>(l) * p.rho_ref * (T_lat - 1.0 / 3.0));
    sg += (double)(float)(w * p.rho_ref * p.T_ref + bg<double>(l) * (p.rho_kappa - p.rho_ref) * p.T_ref);
  }
  d.Fref = dev ? (float)sf : 0.f;
  d.Gref = dev ? (float)sg : 0.f;
  d.wet_d = p.rho_wall_d > 0.0 ? 1 : 0;
  d.wet_u = p.rho_wall_u > 0.0 ? 1 : 0;
  d.psi_form = p.psi_form;
  auto psi_host = [&](double r) { return p.psi_form ? 1.0 - exp(-r) : exp(-1.0 / r); };
  d.psi_wd = d.wet_d ? (float)psi_host(p.rho_wall_d) : 0.f;
  d.psi_wu = d.wet_u ? (float)psi_host(p.rho_wall_u) : 0.f;
  d.one = 1.f;
  return d;
}

// Tile shapes of the pipelined kernel: f(TX, TY) with integral constants.
template <typename F>
int with_pipe_tile(int tx, int ty, F&& f) {
  using std::integral_constant;
  if (tx == 32 && ty == 16) return f(integral_constant<int, 32>{}, integral_constant<int, 16>{});
  if (tx == 32 && ty == 8) return f(integral_constant<int, 32>{}, integral_constant<int, 8>{});
  if (tx == 64 && ty == 8) return f(integral_constant<int, 64>{}, integral_constant<int, 8>{});
  if (tx == 16 && ty == 16) return f(integral_constant<int, 16>{}, integral_constant<int, 16>{});
  if (tx == 128 && ty == 4) return f(integral_constant<int, 128>{}, integral_constant<int, 4>{});
  if (tx == 256 && ty == 2) return f(integral_constant<int, 256>{}, integral_constant<int, 2>{});
  return fail(LBM_EINVAL, "unsupported tile shape for the pipelined kernel");
}

template <typename C>
int launch_pipe(lbm_handle* h, const void* in, void* out) {
  if constexpr (std::is_same<C, F64>::value) {
    return fail(LBM_EINVAL, "the pipelined kernel is built for FP32 and the 16-bit forms only");
  } else {
    const pipe::PParams P = pipe_params(h->p);
    return with_pipe_tile(h->tile_x, h->tile_y, [&](auto X, auto Y) -> int {
      constexpr int TX = decltype(X)::value, TY = decltype(Y)::value;
      const int ntx = (h->p.nx + TX - 1) / TX, nty = (h->p.ny + TY - 1) / TY;
      const int kz = h->z_chunk;
      const int nzc = (h->p.nz + kz - 1) / kz;
      const long long nblk = (long long)ntx * nty * nzc;
      if (nblk > 0x7fffffffLL) return fail(LBM_EINVAL, "grid too large");
      hipLaunchKernelGGL((pipe::k_pipe<C, TX, TY>), dim3((unsigned)nblk), dim3(TX * TY), 0,
                         h->stream, (const char*)in, (char*)out, P, ntx, nty, kz);
      HIP_TRY(hipGetLastError());
      return (int)LBM_OK;
    });
  }
}

template <typename C>
int pipe_groups_per_cu(int tx, int ty) {
  if constexpr (std::is_same<C, F64>::value) {
    return 0;
  } else {
    return with_pipe_tile(tx, ty, [&](auto X, auto Y) -> int {
      constexpr int TX = decltype(X)::value, TY = decltype(Y)::value;
      int nb = 0;
      if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, pipe::k_pipe<C, TX, TY>, TX * TY, 0) !=
          hipSuccess)
        return 0;
      return nb;
    });
  }
}

template <typename C>
int launch_rhoE(lbm_handle* h, const void* in) {
  using R = typename C::R;
  const DevParams<R> P = dev_params<R>(h->p);
  hipLaunchKernelGGL((k_rhoE<C>), dim3(grid_for(h->L.N, 256)), dim3(256), 0, h->stream,
                     (const typename C::S*)in, (R*)h->srho, (R*)h->sE, (R*)h->spsi, P);
  HIP_TRY(hipGetLastError());
  return LBM_OK;
}

// rho and E of the current state in srho / sE, computed once per state
// (diagnostics of one state share them)
template <typename C>
int current_rhoE(lbm_handle* h) {
  if (h->rhoE_version == h->state_version) return LBM_OK;
  const int rc = launch_rhoE<C>(h, h->buf[h->cur]);
  if (rc == LBM_OK) h->rhoE_version = h->state_version;
  return rc;
}

template <typename C>
int launch_reference(lbm_handle* h, const void* in, void* out) {
  using R = typename C::R;
  int rc = launch_rhoE<C>(h, in);
  if (rc) return rc;
  const DevParams<R> P = dev_params<R>(h->p);
  hipLaunchKernelGGL((k_collide<C>), dim3(grid_for(h->L.N, 256)), dim3(256), 0, h->stream,
                     (const typename C::S*)in, (typename C::S*)out, (const R*)h->srho,
                     (const R*)h->sE, (const R*)h->spsi, P);
  HIP_TRY(hipGetLastError());
  return LBM_OK;
}

template <typename C>
int do_step(lbm_handle* h) {
  const void* in = h->buf[h->cur];
  void* out = h->buf[1 - h->cur];
  int rc;
  switch (h->kernel) {
    case LBM_KERNEL_FUSED: rc = launch_fused<C, true>(h, in, out); break;
    case LBM_KERNEL_FUSED_RELOAD: rc = launch_fused<C, false>(h, in, out); break;
    case LBM_KERNEL_PIPELINED: rc = launch_pipe<C>(h, in, out); break;
    default: rc = launch_reference<C>(h, in, out); break;
  }
  if (rc) return rc;
  h->cur = 1 - h->cur;
  h->t += 1;
  ++h->state_version;
  return LBM_OK;
}

template <typename C>
int do_init(lbm_handle* h, const double* rho0, const double* T0) {
  using R = typename C::R;
  const DevParams<R> P = dev_params<R>(h->p);
  hipLaunchKernelGGL((k_init<C>), dim3(grid_for(h->L.N, 256)), dim3(256), 0, h->stream,
                     (typename C::S*)h->buf[0], rho0, T0, P);
  HIP_TRY(hipGetLastError());
  return LBM_OK;
}

template <typename C>
int do_get(lbm_handle* h, double* st) {
  using R = typename C::R;
  const DevParams<R> P = dev_params<R>(h->p);
  hipLaunchKernelGGL((k_get_state<C>), dim3(grid_for(h->L.N, 256)), dim3(256), 0,
                     h->stream, (const typename C::S*)h->buf[h->cur], st, P);
  HIP_TRY(hipGetLastError());
  return LBM_OK;
}

template <typename C>
int do_set(lbm_handle* h, const double* st) {
  using R = typename C::R;
  const DevParams<R> P = dev_params<R>(h->p);
  hipLaunchKernelGGL((k_set_state<C>), dim3(grid_for(h->L.N, 256)), dim3(256), 0,
                     h->stream, (typename C::S*)h->buf[h->cur], st, P);
  HIP_TRY(hipGetLastError());
  return LBM_OK;
}

template <typename C>
int do_moments(lbm_handle* h, double* totals, double* fields) {
  using R = typename C::R;
  int rc = current_rhoE<C>(h);
  if (rc) return rc;
  const DevParams<R> P = dev_params<R>(h->p);
  const int nblk = std::min(kDiagBlocks, grid_for(h->L.N, 256));
  hipLaunchKernelGGL((k_diag<C>), dim3(nblk), dim3(256), 0, h->stream,
                     (const typename C::S*)h->buf[h->cur], (const R*)h->srho, (const R*)h->sE,
                     (const R*)h->spsi, P,
                     h->p.c_v, h->p.G, fields, h->partials);
  HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(k_finish_totals, dim3(1), dim3(256), 0, h->stream, h->partials, nblk, h->small);
  HIP_TRY(hipGetLastError());
  double out[7];
  HIP_TRY(hipMemcpyAsync(out, h->small, sizeof(out), hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(hipStreamSynchronize(h->stream));
  if (totals)
    for (int q = 0; q < 6; ++q) totals[q] = out[q];
  if (out[6] != 0.0) return fail(LBM_ENUMERIC, "non-finite value or rho <= 0 in the state");
  return LBM_OK;
}

template <typename C>
int do_nusselt(lbm_handle* h, double* nb, double* nt, double* nu_z, double* T_z) {
  using R = typename C::R;
  int rc = current_rhoE<C>(h);
  if (rc) return rc;
  const DevParams<R> P = dev_params<R>(h->p);
  // slices per plane: about 1536 work-groups in all (two rounds of three
  // 256-thread groups per CU on 256 CUs), no more slices than 256-node
  // strips of a plane, and the slice sums must fit the partials buffer;
  // the count depends on the shape only, so the sums' order does too
  const int nz = h->p.nz, plane = h->p.nx * h->p.ny;
  int S = 1;
  if (2LL * nz <= 8LL * kDiagBlocks)
    S = std::max(1, std::min({(1536 + nz - 1) / nz, (plane + 255) / 256, (4 * kDiagBlocks) / nz}));
  hipLaunchKernelGGL((k_plane<C>), dim3(nz * S), dim3(256), 0, h->stream,
                     (const typename C::S*)h->buf[h->cur], (const R*)h->srho, (const R*)h->sE,
                     (const R*)h->spsi, P,
                     h->p.c_v, h->p.G, S, S == 1 ? h->prof : h->partials);
  HIP_TRY(hipGetLastError());
  if (S > 1) {
    hipLaunchKernelGGL(k_plane_sum, dim3(grid_for(nz, 256)), dim3(256), 0, h->stream, h->partials, S,
                       nz, plane, h->prof);
    HIP_TRY(hipGetLastError());
  }
  const double kappa = h->p.c_v * (h->p.tau_kappa - 0.5) * h->p.rho_kappa / 3.0;
  hipLaunchKernelGGL(k_finish_nusselt, dim3(1), dim3(256), 0, h->stream, h->prof, h->p.nz,
                     h->p.T_d, h->p.T_u, kappa, h->small);
  HIP_TRY(hipGetLastError());
  double* host = (double*)malloc(sizeof(double) * (2 + 2 * (size_t)nz));
  if (!host) return fail(LBM_EINVAL, "host allocation failed");
  hipError_t e = hipMemcpyAsync(host, h->small, sizeof(double) * (2 + 2 * (size_t)nz),
                                hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) {
    free(host);
    return fail(LBM_EHIP, std::string("nusselt copy: ") + hipGetErrorString(e));
  }
  if (nb) *nb = host[0];
  if (nt) *nt = host[1];
  if (nu_z) memcpy(nu_z, host + 2, sizeof(double) * nz);
  if (T_z) memcpy(T_z, host + 2 + nz, sizeof(double) * nz);
  free(host);
  return LBM_OK;
}

template <typename C>
int do_hist(lbm_handle* h, const HistSpec& hs, unsigned long long* counts, double* sums,
            uint64_t* out_of_range) {
  using R = typename C::R;
  int rc = current_rhoE<C>(h);
  if (rc) return rc;
  const DevParams<R> P = dev_params<R>(h->p);
  const size_t nbins = (size_t)hs.nxb * hs.nyb;
  hipLaunchKernelGGL(k_zero_u64, dim3(grid_for(nbins, 256)), dim3(256), 0, h->stream, counts, nbins);
  HIP_TRY(hipGetLastError());
  const size_t nodes = (size_t)(hs.k1 - hs.k0) * h->p.nx * h->p.ny;
  const int nblk = std::max(1, std::min(kDiagBlocks, grid_for(nodes, 256)));
  const size_t lds = nbins <= (size_t)kLdsBins ? nbins * sizeof(uint32_t) : 0;
  hipLaunchKernelGGL((k_hist<C>), dim3(nblk), dim3(256), lds, h->stream,
                     (const typename C::S*)h->buf[h->cur], (const R*)h->srho, (const R*)h->sE,
                     (const R*)h->spsi, P,
                     h->p.c_v, h->p.G, hs, counts, h->partials);
  HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(k_finish_totals, dim3(1), dim3(256), 0, h->stream, h->partials, nblk, h->small);
  HIP_TRY(hipGetLastError());
  double out[7];
  HIP_TRY(hipMemcpyAsync(out, h->small, sizeof(out), hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(hipStreamSynchronize(h->stream));
  if (sums)
    for (int q = 0; q < 5; ++q) sums[q] = out[q];
  if (out_of_range) *out_of_range = (uint64_t)out[5];
  return LBM_OK;
}

constexpr int kIncBlocks = 1024;

template <typename C>
int do_structure(lbm_handle* h, int k0, int k1, int which, int rmax, double* work, double* out) {
  using R = typename C::R;
  int rc = current_rhoE<C>(h);
  if (rc) return rc;
  const DevParams<R> P = dev_params<R>(h->p);
  const int nx = h->p.nx, ny = h->p.ny, planes = k1 - k0;
  const size_t nodes = (size_t)planes * nx * ny;
  hipLaunchKernelGGL((k_quantity<C>), dim3(std::min(kDiagBlocks, grid_for(nodes, 256))), dim3(256),
                     0, h->stream, (const typename C::S*)h->buf[h->cur], (const R*)h->srho,
                     (const R*)h->sE, (const R*)h->spsi, P, h->p.c_v, h->p.G, k0, k1, which, work);
  HIP_TRY(hipGetLastError());
  double* part = work + nodes;
  double* sums = part + (size_t)kIncBlocks * rmax * 2;
  const size_t lds = (size_t)std::max(nx, ny) * sizeof(double);
  hipLaunchKernelGGL(k_increments, dim3(kIncBlocks), dim3(256), lds, h->stream, work, nx, ny,
                     planes, rmax, part);
  HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(k_finish_increments, dim3(1), dim3(256), 0, h->stream, part, kIncBlocks, rmax,
                     sums);
  HIP_TRY(hipGetLastError());
  double host[2 * 256];   // r_max <= 256 (checked by the entry points)
  HIP_TRY(hipMemcpyAsync(host, sums, sizeof(double) * 2 * rmax, hipMemcpyDeviceToHost,
                         h->stream));
  HIP_TRY(hipStreamSynchronize(h->stream));
  // each separation is counted once per node and direction
  const double cnt = 2.0 * (double)nodes;
  for (int r = 0; r < rmax; ++r) {
    out[r] = host[2 * r] / cnt;
    out[rmax + r] = host[2 * r + 1] / cnt;
  }
  return LBM_OK;
}

template <typename R>
int do_adjoint_step(lbm_handle* h, const double* st, const double* lam1, double* lam0,
                    double* grads) {
  const DevParams<R> P = dev_params<R>(h->p);
  const size_t N = h->L.N;
  hipLaunchKernelGGL((k_adj_rhoE<R>), dim3(grid_for(N, 256)), dim3(256), 0, h->stream, st,
                     (R*)h->arho, (R*)h->aE, P);
  HIP_TRY(hipGetLastError());
  const int nblk = std::min(kDiagBlocks, grid_for(N, 256));
  hipLaunchKernelGGL((k_adj_local<R>), dim3(nblk), dim3(256), 0, h->stream, st, lam1, lam0,
                     (const R*)h->arho, (const R*)h->aE, (R*)h->gbar, P, h->partials);
  HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL((k_adj_stencil<R>), dim3(grid_for(N, 256)), dim3(256), 0, h->stream,
                     (const R*)h->arho, (const R*)h->gbar, lam0, P);
  HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(k_finish_totals, dim3(1), dim3(256), 0, h->stream, h->partials, nblk, h->small);
  HIP_TRY(hipGetLastError());
  double out[2];
  HIP_TRY(hipMemcpyAsync(out, h->small, sizeof(out), hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(hipStreamSynchronize(h->stream));
  if (grads) {
    grads[0] += out[0];
    grads[1] += out[1];
  }
  return LBM_OK;
}

template <typename R>
int do_adjoint_qbot(lbm_handle* h, const double* st, double weight, double* lam, double* q,
                    double* grads) {
  const DevParams<R> P = dev_params<R>(h->p);
  const size_t A = (size_t)h->p.nx * h->p.ny;
  const int nblk = std::min(kDiagBlocks, grid_for(A, 256));
  const double kappa = h->p.c_v * (h->p.tau_kappa - 0.5) * h->p.rho_kappa / 3.0;
  hipLaunchKernelGGL((k_adj_qbot<R>), dim3(nblk), dim3(256), 0, h->stream, st, lam, P, weight,
                     kappa, h->partials);
  HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(k_finish_totals, dim3(1), dim3(256), 0, h->stream, h->partials, nblk, h->small);
  HIP_TRY(hipGetLastError());
  double sumT;
  HIP_TRY(hipMemcpyAsync(&sumT, h->small, sizeof(double), hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(hipStreamSynchronize(h->stream));
  if (q) *q = 2.0 * kappa * (h->p.T_d - sumT / (double)A);
  if (grads) grads[1] += weight * 2.0 * kappa;
  return LBM_OK;
}

template <typename R>
int do_adjoint_init(lbm_handle* h, const double* lam0, const double* T0, double* out) {
  const DevParams<R> P = dev_params<R>(h->p);
  hipLaunchKernelGGL((k_adj_init<R>), dim3(grid_for(h->L.N, 256)), dim3(256), 0, h->stream,
                     lam0, T0, out, P);
  HIP_TRY(hipGetLastError());
  return LBM_OK;
}

template <template <typename> class Fn, typename... A>
int dispatch(int storage, A... a) {
  switch (storage) {
    case LBM_FP64: return Fn<F64>::run(a...);
    case LBM_FP32: return Fn<F32>::run(a...);
    case LBM_FP16DEV: return Fn<H16>::run(a...);
    default: return Fn<B16>::run(a...);
  }
}
template <typename C> struct StepFn { static int run(lbm_handle* h) { return do_step<C>(h); } };
template <typename C> struct OccupancyFn {
  static int run(int kernel, int tx, int ty) {
    if (kernel == LBM_KERNEL_PIPELINED) return pipe_groups_per_cu<C>(tx, ty);
    return kernel == LBM_KERNEL_FUSED_RELOAD ? fused_groups_per_cu<C, false>(tx, ty)
                                             : fused_groups_per_cu<C, true>(tx, ty);
  }
};
template <typename C> struct InitFn {
  static int run(lbm_handle* h, const double* r, const double* T) { return do_init<C>(h, r, T); }
};
template <typename C> struct GetFn { static int run(lbm_handle* h, double* s) { return do_get<C>(h, s); } };
template <typename C> struct SetFn {
  static int run(lbm_handle* h, const double* s) { return do_set<C>(h, s); }
};
template <typename C> struct MomFn {
  static int run(lbm_handle* h, double* t, double* f) { return do_moments<C>(h, t, f); }
};
template <typename C> struct HistFn {
  static int run(lbm_handle* h, HistSpec hs, unsigned long long* c, double* s, uint64_t* o) {
    return do_hist<C>(h, hs, c, s, o);
  }
};
template <typename C> struct SfFn {
  static int run(lbm_handle* h, int k0, int k1, int q, int rmax, double* w, double* o) {
    return do_structure<C>(h, k0, k1, q, rmax, w, o);
  }
};
template <typename C> struct CheckFn {
  static int run(lbm_handle* h, double* out) {
    using R = typename C::R;
    const DevParams<R> P = dev_params<R>(h->p);
    const int nblk = std::min(kDiagBlocks, grid_for(h->L.N, 256));
    hipLaunchKernelGGL((k_check<C>), dim3(nblk), dim3(256), 0, h->stream,
                       (const typename C::S*)h->buf[h->cur], P, h->partials);
    HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_finish_totals, dim3(1), dim3(256), 0, h->stream, h->partials, nblk, h->small);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(out, h->small, 3 * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    return LBM_OK;
  }
};
template <typename C> struct PworkFn {
  static int run(lbm_handle* h, double* work, double* out) {
    double tot[6];
    int rc = do_moments<C>(h, tot, work);
    if (rc) return rc;
    hipLaunchKernelGGL(k_pwork, dim3(h->p.nz), dim3(256), 0, h->stream, work, h->p.nx, h->p.ny,
                       h->p.nz, h->p.periodic_z ? 1 : 0, h->p.G, h->p.psi_form, h->prof);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(out, h->prof, sizeof(double) * (size_t)h->p.nz, hipMemcpyDeviceToHost,
                           h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    return LBM_OK;
  }
};
template <typename C> struct NuFn {
  static int run(lbm_handle* h, double* a, double* b, double* c, double* d) {
    return do_nusselt<C>(h, a, b, c, d);
  }
};

}  // namespace

extern "C" {

const char* lbm_version(void) { return "paper_1111_0905_amd lbm 0.1 (gfx950)"; }

const char* lbm_last_error(void) { return g_err.c_str(); }

size_t lbm_workspace_bytes(const lbm_params* p) {
  if (validate(p) != LBM_OK) return 0;
  return layout(p).total;
}

int lbm_seeded_density(int32_t nx, int32_t ny, int32_t nz, uint64_t seed, double rho_mean,
                       double noise_amp, double* rho0, void* stream) {
  if (!rho0) return fail(LBM_EINVAL, "rho0 is NULL");
  if (nx < 1 || ny < 1 || nz < 1) return fail(LBM_EINVAL, "nx, ny, nz must be >= 1");
  if (!(rho_mean > 0.0) || !(noise_amp >= 0.0) || !(noise_amp < 1.0))
    return fail(LBM_EINVAL, "need rho_mean > 0 and 0 <= noise_amp < 1");
  const size_t N = (size_t)nx * ny * nz;
  hipLaunchKernelGGL(k_seeded_density, dim3(grid_for(N, 256)), dim3(256), 0,
                     (hipStream_t)stream, rho0, N, seed, rho_mean, noise_amp);
  HIP_TRY(hipGetLastError());
  return LBM_OK;
}

int lbm_init(const lbm_params* p, void* workspace, size_t workspace_bytes, const double* rho0,
             const double* T0, void* stream, lbm_handle** out) {
  g_err.clear();
  if (!out) return fail(LBM_EINVAL, "out is NULL");
  *out = nullptr;
  int rc = validate(p);
  if (rc) return rc;
  if (!rho0) return fail(LBM_EINVAL, "rho0 is NULL");
  const Layout L = layout(p);
  if (!workspace || workspace_bytes < L.total)
    return fail(LBM_EWORKSPACE, "workspace smaller than lbm_workspace_bytes()");
  if (((uintptr_t)workspace) % kAlign)
    return fail(LBM_EWORKSPACE, "workspace must be 256-byte aligned");
  lbm_handle* h = new (std::nothrow) lbm_handle();
  if (!h) return fail(LBM_EINVAL, "host allocation failed");
  h->p = *p;
  h->L = L;
  h->stream = (hipStream_t)stream;
  h->ws = (char*)workspace;
  char* c = h->ws;
  h->buf[0] = c; c += L.buf;
  h->buf[1] = c; c += L.buf;
  h->srho = c; c += L.scr;
  h->sE = c; c += L.scr;
  h->spsi = c; c += L.scr;
  h->partials = (double*)c; c += L.part;
  h->small = (double*)c; c += L.small;
  h->prof = (double*)c; c += L.small;
  h->gbar = L.adj ? (double*)c : nullptr;
  h->arho = L.adj ? h->gbar + 9 * L.N : nullptr;
  h->aE = L.adj ? h->gbar + 10 * L.N : nullptr;
  h->cur = 0;
  h->t = 0;
  h->state_version = 1;
  h->rhoE_version = 0;
  // defaults from tile/variant sweeps on MI355X (same process, alternating):
  // FP32 and the 16-bit forms use the pipelined kernel on 512-thread tiles
  // as wide as the plane allows (128 x 4: 512^3 FP32 9.14 ms, 256^3 -10 %,
  // 128^3 -12 % against the register-resident kernel on 32 x 16 / 64 x 8;
  // FP16 512^3 5.59 ms against 6.74 ms re-reading on 64 x 16; wider rows
  // mean fewer cache lines shared with the x-neighbour tiles and fewer
  // scattered side-ring loads); FP64 keeps the register-resident kernel on
  // 64 x 2 tiles
  int cus = 0, dev = 0;  // compute units of the current device
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      cus < 1)
    cus = 256;
  h->dev = dev;
  {
    // this device's copy of the static scratch (once per device, with the
    // device current)
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (dev >= 0 && dev < kMaxDevices && !g_scratch_ptr[dev]) {
      void* ptr = nullptr;
      const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
      if (e != hipSuccess || !ptr) {
        delete h;
        return fail(LBM_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
      }
      g_scratch_ptr[dev] = (double*)ptr;
    }
  }
  h->kernel = p->kernel;
  const int wide_x = p->nx >= 128 ? 128 : (p->nx >= 64 ? 64 : 32);
  if (p->kernel == LBM_KERNEL_PIPELINED) {
    h->tile_x = p->tile_x ? p->tile_x : wide_x;
    h->tile_y = p->tile_y ? p->tile_y : 512 / h->tile_x;
  } else if (p->tile_x == 0 && p->tile_y == 0) {
    if (p->storage == LBM_FP64) {
      h->tile_x = 64;
      h->tile_y = 2;
    } else if (p->kernel == LBM_KERNEL_FUSED) {
      h->kernel = LBM_KERNEL_PIPELINED;
      h->tile_x = wide_x;
      h->tile_y = 512 / wide_x;
    } else if (p->storage == LBM_FP32) {
      const bool wide = (long long)p->nx * p->ny >= 2LL * cus * 32 * 16;
      h->tile_x = wide ? 32 : 64;
      h->tile_y = wide ? 16 : 8;
    } else {
      h->tile_x = 64;
      h->tile_y = 16;
    }
  } else {
    h->tile_x = p->tile_x ? p->tile_x : 64;
    h->tile_y = p->tile_y ? p->tile_y : 8;
  }
  if (p->z_chunk) {
    h->z_chunk = std::min(p->z_chunk, p->nz);
  } else {
    // split the z columns into the number of chunks that makes the launch
    // shortest: its rounds of resident work-groups (compute units x
    // work-groups per unit for this kernel) times the planes each work-group
    // marches (its chunk and the halo plane it re-reads on each side).  One
    // chunk when the tiles fill whole rounds; a split when one round would
    // not fill the GPU or the last round would run nearly empty.  Chunks stay
    // at least 4 planes deep; ties go to fewer chunks.
    const long long tiles = (long long)((p->nx + h->tile_x - 1) / h->tile_x) *
                            ((p->ny + h->tile_y - 1) / h->tile_y);
    int per_cu = h->kernel == LBM_KERNEL_REFERENCE
                     ? 1
                     : dispatch<OccupancyFn>(p->storage, h->kernel, h->tile_x, h->tile_y);
    if (per_cu < 1) per_cu = 1;
    const long long want = (long long)cus * per_cu;
    int zc_best = p->nz;
    long long cost_best = -1;
    for (int c = 1; c <= p->nz; ++c) {
      const int zc = (p->nz + c - 1) / c;
      if (c > 1 && zc < 4) break;
      if (c > 1 && zc == (p->nz + c - 2) / (c - 1)) continue;   // same chunks as c - 1
      const long long chunks = (p->nz + zc - 1) / zc;
      const long long cost = (tiles * chunks + want - 1) / want * (zc + 2);
      if (cost_best < 0 || cost < cost_best) {
        cost_best = cost;
        zc_best = zc;
      }
    }
    h->z_chunk = std::min(zc_best, p->nz);
  }
  rc = dispatch<InitFn>(p->storage, h, rho0, T0);
  if (rc == LBM_OK) {
    hipError_t e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) rc = fail(LBM_EHIP, std::string("init: ") + hipGetErrorString(e));
  }
  if (rc) {
    delete h;
    return rc;
  }
  *out = h;
  return LBM_OK;
}

int lbm_step(lbm_handle* h, int64_t n) {
  if (!h) return fail(LBM_EINVAL, "handle is NULL");
  if (n < 0) return fail(LBM_EINVAL, "n must be >= 0");
  for (int64_t s = 0; s < n; ++s) {
    int rc = dispatch<StepFn>(h->p.storage, h);
    if (rc) return rc;
    if (h->check_every > 0 && h->t % h->check_every == 0) {
      double c[3];
      rc = dispatch<CheckFn>(h->p.storage, h, c);
      if (rc) return rc;
      if (c[2] != 0.0)
        return fail(LBM_ENUMERIC, "step " + std::to_string(h->t) + ": " +
                                      std::to_string((long long)c[2]) +
                                      " nodes with non-finite populations or rho <= 0");
      if (h->check_mass0 == 0.0) {
        h->check_mass0 = c[0];
      } else if (!(std::fabs(c[0] / h->check_mass0 - 1.0) <= h->check_mass_tol)) {
        return fail(LBM_ENUMERIC, "step " + std::to_string(h->t) + ": stored mass changed by " +
                                      std::to_string(c[0] / h->check_mass0 - 1.0) +
                                      " (relative)");
      }
    }
  }
  return LBM_OK;
}

int lbm_set_check(lbm_handle* h, int64_t every, double mass_tol) {
  if (!h) return fail(LBM_EINVAL, "handle is NULL");
  if (every < 0 || !(mass_tol > 0.0)) return fail(LBM_EINVAL, "need every >= 0 and mass_tol > 0");
  h->check_every = every;
  h->check_mass_tol = mass_tol;
  h->check_mass0 = 0.0;
  return LBM_OK;
}

int64_t lbm_time(const lbm_handle* h) { return h ? h->t : -1; }

int lbm_moments(lbm_handle* h, double* totals, double* fields) {
  if (!h) return fail(LBM_EINVAL, "handle is NULL");
  return dispatch<MomFn>(h->p.storage, h, totals, fields);
}

int lbm_nusselt(lbm_handle* h, double* nu_bot, double* nu_top, double* nu_z, double* T_z) {
  if (!h) return fail(LBM_EINVAL, "handle is NULL");
  if (h->p.periodic_z) return fail(LBM_EINVAL, "Nusselt numbers need walls");
  if (!(h->p.T_d != h->p.T_u)) return fail(LBM_EINVAL, "Nusselt numbers need T_d != T_u");
  return dispatch<NuFn>(h->p.storage, h, nu_bot, nu_top, nu_z, T_z);
}

int lbm_pressure_work(lbm_handle* h, double* work, size_t work_bytes, double* pw_z) {
  if (!h || !work || !pw_z) return fail(LBM_EINVAL, "NULL argument");
  if (work_bytes < 5 * h->L.N * sizeof(double))
    return fail(LBM_EWORKSPACE, "work buffer smaller than 5 * nx * ny * nz doubles");
  return dispatch<PworkFn>(h->p.storage, h, work, pw_z);
}

int lbm_histogram(lbm_handle* h, int32_t k0, int32_t k1, int32_t qx, double x_lo, double x_hi,
                  int32_t nx_bins, int32_t qy, double y_lo, double y_hi, int32_t ny_bins,
                  uint64_t* counts, uint64_t* out_of_range, double* sums) {
  if (!h || !counts) return fail(LBM_EINVAL, "NULL argument");
  if (k0 < 0 || k1 > h->p.nz || k0 >= k1) return fail(LBM_EINVAL, "need 0 <= k0 < k1 <= nz");
  if (qx < LBM_Q_RHO || qx > LBM_Q_HEATFLUX || qy < -1 || qy > LBM_Q_HEATFLUX)
    return fail(LBM_EINVAL, "unknown quantity");
  if (nx_bins < 1 || ny_bins < 1 || (qy < 0 && ny_bins != 1))
    return fail(LBM_EINVAL, "bins must be >= 1 (ny_bins = 1 for a 1-D histogram)");
  if ((double)nx_bins * (double)ny_bins > 67108864.0) return fail(LBM_EINVAL, "too many bins");
  if (!(x_hi > x_lo) || (qy >= 0 && !(y_hi > y_lo))) return fail(LBM_EINVAL, "empty bin range");
  HistSpec hs;
  hs.k0 = k0;
  hs.k1 = k1;
  hs.qx = qx;
  hs.qy = qy;
  hs.nxb = nx_bins;
  hs.nyb = ny_bins;
  hs.xlo = x_lo;
  hs.xscale = (double)nx_bins / (x_hi - x_lo);
  hs.ylo = qy >= 0 ? y_lo : 0.0;
  hs.yscale = qy >= 0 ? (double)ny_bins / (y_hi - y_lo) : 1.0;
  return dispatch<HistFn>(h->p.storage, h, hs, (unsigned long long*)counts, sums, out_of_range);
}

size_t lbm_structure_work_bytes(const lbm_handle* h, int32_t k0, int32_t k1, int32_t r_max) {
  if (!h || k0 < 0 || k1 > h->p.nz || k0 >= k1 || r_max < 1) return 0;
  return sizeof(double) * ((size_t)(k1 - k0) * h->p.nx * h->p.ny +
                           (size_t)kIncBlocks * r_max * 2 + 2 * (size_t)r_max);
}

int lbm_structure_functions(lbm_handle* h, int32_t k0, int32_t k1, int32_t q, int32_t r_max,
                            double* work, size_t work_bytes, double* out) {
  if (!h || !work || !out) return fail(LBM_EINVAL, "NULL argument");
  if (k0 < 0 || k1 > h->p.nz || k0 >= k1) return fail(LBM_EINVAL, "need 0 <= k0 < k1 <= nz");
  if (q < LBM_Q_RHO || q > LBM_Q_HEATFLUX) return fail(LBM_EINVAL, "unknown quantity");
  if (r_max < 1 || r_max > 256 || r_max >= h->p.nx || r_max >= h->p.ny)
    return fail(LBM_EINVAL, "need 1 <= r_max <= 256 and r_max < nx, ny");
  if ((size_t)std::max(h->p.nx, h->p.ny) * sizeof(double) > 65536)
    return fail(LBM_EINVAL, "lines longer than 8192 nodes are not supported");
  if (work_bytes < lbm_structure_work_bytes(h, k0, k1, r_max))
    return fail(LBM_EWORKSPACE, "work buffer too small (lbm_structure_work_bytes)");
  return dispatch<SfFn>(h->p.storage, h, (int)k0, (int)k1, (int)q, (int)r_max, work, out);
}

int lbm_structure_functions_noalloc(lbm_handle* h, int32_t k0, int32_t k1, int32_t q,
                                    int32_t r_max, double* out) {
  if (!h || !out) return fail(LBM_EINVAL, "NULL argument");
  if (k0 < 0 || k1 > h->p.nz || k0 >= k1) return fail(LBM_EINVAL, "need 0 <= k0 < k1 <= nz");
  if (q < LBM_Q_RHO || q > LBM_Q_HEATFLUX) return fail(LBM_EINVAL, "unknown quantity");
  if (r_max < 1 || r_max > 256 || r_max >= h->p.nx || r_max >= h->p.ny)
    return fail(LBM_EINVAL, "need 1 <= r_max <= 256 and r_max < nx, ny");
  if ((size_t)std::max(h->p.nx, h->p.ny) * sizeof(double) > 65536)
    return fail(LBM_EINVAL, "lines longer than 8192 nodes are not supported");
  const size_t need = lbm_structure_work_bytes(h, k0, k1, r_max);
  if (need > kStaticScratchDoubles * sizeof(double))
    return fail(LBM_EWORKSPACE, "planes k0..k1 need " + std::to_string(need) +
                                    " bytes of scratch, more than the 33554432 bytes of the static "
                                    "scratch: use lbm_structure_functions with a work buffer");
  double* ptr = (h->dev >= 0 && h->dev < kMaxDevices) ? g_scratch_ptr[h->dev] : nullptr;
  if (!ptr) return fail(LBM_EHIP, "no static scratch on the handle's device");
  return dispatch<SfFn>(h->p.storage, h, (int)k0, (int)k1, (int)q, (int)r_max, ptr, out);
}

int lbm_get_state(lbm_handle* h, double* state) {
  if (!h || !state) return fail(LBM_EINVAL, "NULL argument");
  return dispatch<GetFn>(h->p.storage, h, state);
}

int lbm_set_state(lbm_handle* h, const double* state) {
  if (!h || !state) return fail(LBM_EINVAL, "NULL argument");
  const int rc = dispatch<SetFn>(h->p.storage, h, state);
  ++h->state_version;
  if (rc == LBM_OK) {
    h->t = 0;
    h->check_mass0 = 0.0;
  }
  return rc;
}

int lbm_adjoint_step(lbm_handle* h, const double* state, const double* adj_in, double* adj_out,
                     double* grads) {
  if (!h || !state || !adj_in || !adj_out) return fail(LBM_EINVAL, "NULL argument");
  if (!h->gbar) return fail(LBM_EINVAL, "handle was created without adjoint = 1");
  if (adj_in == adj_out) return fail(LBM_EINVAL, "adj_in and adj_out must not alias");
  return do_adjoint_step<double>(h, state, adj_in, adj_out, grads);
}

int lbm_adjoint_qbot(lbm_handle* h, const double* state, double weight, double* adj, double* q,
                     double* grads) {
  if (!h || !state) return fail(LBM_EINVAL, "NULL argument");
  if (h->p.periodic_z) return fail(LBM_EINVAL, "the wall heat flux needs walls");
  return do_adjoint_qbot<double>(h, state, weight, adj, q, grads);
}

int lbm_adjoint_init_rho(lbm_handle* h, const double* adj0, const double* T0, double* dJ_drho0) {
  if (!h || !adj0 || !dJ_drho0) return fail(LBM_EINVAL, "NULL argument");
  return do_adjoint_init<double>(h, adj0, T0, dJ_drho0);
}

int lbm_stream_copy(const void* src, void* dst, size_t bytes, int32_t nontemporal, void* stream) {
  if (!src || !dst) return fail(LBM_EINVAL, "NULL argument");
  if (bytes == 0 || bytes % 16 || ((uintptr_t)src | (uintptr_t)dst) % 16)
    return fail(LBM_EINVAL, "bytes must be a positive multiple of 16 and both pointers 16-byte aligned");
  const size_t n = bytes / 16;
  const size_t grid = (n + 255) / 256;
  if (grid > 0x7fffffffULL) return fail(LBM_EINVAL, "copy too large");
  if (nontemporal)
    hipLaunchKernelGGL(k_copy16<true>, dim3((unsigned)grid), dim3(256), 0, (hipStream_t)stream,
                       (const float4*)src, (float4*)dst, n);
  else
    hipLaunchKernelGGL(k_copy16<false>, dim3((unsigned)grid), dim3(256), 0, (hipStream_t)stream,
                       (const float4*)src, (float4*)dst, n);
  HIP_TRY(hipGetLastError());
  return LBM_OK;
}

int lbm_stream_rows(const void* src, void* dst, int32_t rows, size_t row_stride, size_t row_bytes,
                    void* stream) {
  if (!src || !dst) return fail(LBM_EINVAL, "NULL argument");
  if (rows != 1 && rows != 2 && rows != 4 && rows != 19)
    return fail(LBM_EINVAL, "rows must be 1, 2, 4 or 19");
  if (row_bytes == 0 || row_bytes % 8 || row_stride % 8 || row_stride < row_bytes ||
      ((uintptr_t)src | (uintptr_t)dst) % 8)
    return fail(LBM_EINVAL, "row_bytes > 0, row_bytes and row_stride multiples of 8, row_stride >= "
                            "row_bytes, pointers 8-byte aligned");
  const size_t n = row_bytes / 8;
  const size_t grid = (n + 255) / 256;
  if (grid > 0x7fffffffULL) return fail(LBM_EINVAL, "rows too long");
  auto go = [&](auto R) {
    hipLaunchKernelGGL((k_rows<decltype(R)::value>), dim3((unsigned)grid), dim3(256), 0,
                       (hipStream_t)stream, (const char*)src, (char*)dst, row_stride, n);
  };
  switch (rows) {
    case 1: go(std::integral_constant<int, 1>{}); break;
    case 2: go(std::integral_constant<int, 2>{}); break;
    case 4: go(std::integral_constant<int, 4>{}); break;
    default: go(std::integral_constant<int, 19>{}); break;
  }
  HIP_TRY(hipGetLastError());
  return LBM_OK;
}

void lbm_destroy(lbm_handle* h) { delete h; }

}  // extern "C"
