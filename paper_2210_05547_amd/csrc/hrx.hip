// hrx: HIP kernels for gfx950 and the C-ABI of include/hrx.h.
//
// One right-hand-side evaluation (Eqs. 5-6 with the sponge of Eq. 26) runs as
//   k_prim     pointwise: Q -> velocities, T (Newton, Sec. 3.4), p, X_s, mu, kappa,
//              D_s (Eq. 19), wdot_s (Eqs. 13-15), h_s, and the AD sources e, Y_s
//              [FP64-ALU bound]
//   k_ad_src, k_ad_march, k_ad_filter_z
//              artificial diffusivity (Sec. 3.3 reading): |S| and theta, fourth
//              differences and the separable 9-point Gaussian filter (x and y in a
//              march down y, z in a march along z)  [HBM / latency bound]
//   k_flux     stencil gradients of u, T, X_s at each point (LDS tiles), then the
//              total flux F_j = F_C,j - F_D,j for every direction j (Eqs. 9, 10, 18)
//              [HBM bound]
//   k_div      -sum_j dF_j/dx_j + S - sigma (Q - Q_ref), boundary rows, and either
//              the R output or the fused low-storage RK update (Sec. 3.1), with the wall
//              condition (no slip, non-catalytic, T_w or adiabatic) in 2-D  [HBM bound]
//   k_bc       the wall row after a 3-D stage
// Fields are SoA planes with x fastest; stencil kernels stage LDS tiles (32 x 8 points
// plus halos) or march along a direction keeping the taps in registers.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <new>
#include <type_traits>
#include <vector>

#include "air5.h"
#include "tpg.h"
#include "hrx.h"
#include "mlp.h"

namespace hrx {

enum { CPG = 0, AIR5 = 1, TPG = 2 };
enum { MODE_RHS = 0, MODE_RK = 1 };
// form of an RK stage's update (Sec. 3.1): two-register low-storage (dQ <- A dQ + dt R,
// Q <- Q + B dQ), or the three-register TVD RK3 with the step's initial state Q0 in dQ
// (first stage: Q0 <- Q; every stage: Q <- A Q0 + B (Q + dt R))
enum { RKF_2N = 0, RKF_SSP_FIRST = 1, RKF_SSP = 2 };

// The update of one value of one component (q: the stage's input state, dq: the second
// register, r: the right-hand side); writes the new state and register through the
// references.  Shared by the fused divergence kernel and the unfused update.  Every
// product and sum is rounded on its own, in the order the stage formulas are written
// (no fused multiply-add): the update then adds no rounding of its own to what the
// right-hand side carries.  The three-register form rounds at the size of the state
// (not of the increment) several times per stage, and on a boundary layer's small
// wall-normal momentum that rounding, not the right-hand side's, decides agreement with
// any other evaluation of the same formulas after many stages.
__device__ __forceinline__ void rk_update(int rkf, double A, double B, double dt, double r,
                                          double q, double dq, double& q_new, double& dq_new,
                                          bool& write_dq) {
#pragma clang fp contract(off)
  if (rkf == RKF_2N) {
    dq_new = A * dq + dt * r;
    q_new = q + B * dq_new;
    write_dq = true;
  } else {
    const double q0 = rkf == RKF_SSP_FIRST ? q : dq;
    q_new = A * q0 + B * (q + dt * r);
    dq_new = q0;
    write_dq = rkf == RKF_SSP_FIRST;
  }
}

// LU factors of one direction's compact-derivative matrix (see k_cd_x, k_cd_col)
struct CLine {
  const double *lo, *up, *iu;   // [n] LU factors (A' for the periodic direction)
  const double* q;              // [n] periodic: A'^-1 u
  double s, alpha;              // periodic: 1/(1 + v.q) and the off-diagonal alpha
};

struct Dev {
  int nx, ny, nz, ndim, nvar, ns, fd_order;
  long N;
  double gamma, Re, Pr, T_ref, mu_inf, kappa_inf, c_inf, rho_inf, L_ref, R_inf;
  // reciprocals and products of the reference values, formed once on the host:
  // 1/T_ref, 1/c_inf^2, (gamma - 1)/(gamma R_inf), 1/mu_inf, 1/kappa_inf,
  // 1/(c_inf L_ref), L_ref/(rho_inf c_inf), 1/c_inf
  double iT_ref, ic2, p_fac, imu_inf, ikappa_inf, iDscale, wscale, ic_inf;
  int wall;
  double T_wall;  // K
  double newton_rtol;
  int newton_max;
  int ad_on;
  double Cmu, Cbeta, Ckap, CD, CY;
  double tpg_k0, tpg_th;          // thermally perfect gas: c_p0 / c_p,inf, Theta / T_ref
  int sm;                         // Stefan-Maxwell diffusion (Eq. 17) instead of Eq. (18)
  int w_iD;                       // Stefan-Maxwell: 10 planes of nondimensional 1/D_sr
  const double *mx, *my, *mz;     // metrics d(xi)/dx
  const double *sx, *sy;          // sponge profiles
  const double *dlx, *dly, *dlz;  // local spacings dx/d(xi)
  const unsigned char *hold;      // [nz][3][nx] or null
  unsigned long long *counters;   // [kind][CSLOTS]: 0 Newton non-converged, 1 below
                                  // e(T_min), 2 surrogate fallbacks, 3 non-finite
                                  // states, 4 negative densities
  // W plane offsets
  int nsrc, w_p, w_mu, w_kap, w_D, w_wdot, w_c;
  int nad;                        // artificial-diffusivity planes (3 + ns)
  int gx;                         // x segments of TX points per grid row
  int tgx, tgy;                   // 2-D LDS tiles per row / column
  int tgz;                        // 3-D (x, z) tiles along z
  int warm;                       // W holds a previous temperature field (Newton warm start)
  int compact;                    // compact first derivatives (gradients from planes)
  CLine cl[3];                    // compact factors of the x, y, z lines
  void* ad;                       // artificial-diffusivity source planes (RT), or null
};

// ------------------------------------------------------------------ stencils
// First derivative in index space along a line of n points with stride s, at
// position i of the line (flat index idx).  Interior: explicit central 6th (or 4th)
// order; ends: one-sided 4th-order closures and their mirror images.  RT is the
// type of the stored plane and of the arithmetic (double, or float in the mixed form).
template <int ORDER, class TA, class TD>
__device__ __forceinline__ TA dline(const TD* __restrict__ f, long idx, long s, int i, int n) {
  // differences are formed in the storage type TD, weighted sums in the arithmetic type TA
  if (ORDER == 6) {
    if (i >= 3 && i <= n - 4) {
      TA acc = TA(0.75) * TA(f[idx + s] - f[idx - s]);
      acc += TA(-0.15) * TA(f[idx + 2 * s] - f[idx - 2 * s]);
      acc += TA(1.0 / 60.0) * TA(f[idx + 3 * s] - f[idx - 3 * s]);
      return acc;
    }
  } else {
    if (i >= 2 && i <= n - 3) {
      TA acc = TA(2.0 / 3.0) * TA(f[idx + s] - f[idx - s]);
      acc += TA(-1.0 / 12.0) * TA(f[idx + 2 * s] - f[idx - 2 * s]);
      return acc;
    }
  }
  // one-sided closures: the weights sum to zero, so subtract the centre value first
  const TD c = f[idx];
  auto df = [&](long o) { return TA(f[idx + o] - c); };
  const TA b01 = TA(4.0), b02 = TA(-3.0), b03 = TA(4.0 / 3.0), b04 = TA(-0.25);
  const TA b10 = TA(-0.25), b12 = TA(1.5), b13 = TA(-0.5), b14 = TA(1.0 / 12.0);
  if (i == 0) return b01 * df(s) + b02 * df(2 * s) + b03 * df(3 * s) + b04 * df(4 * s);
  if (i == 1) return b10 * df(-s) + b12 * df(s) + b13 * df(2 * s) + b14 * df(3 * s);
  if (i == n - 1) return -(b01 * df(-s) + b02 * df(-2 * s) + b03 * df(-3 * s) + b04 * df(-4 * s));
  if (i == n - 2) return -(b10 * df(s) + b12 * df(-s) + b13 * df(-2 * s) + b14 * df(-3 * s));
  // 6th order only: points 2 and n-3 use the central 4th-order stencil
  TA acc = TA(2.0 / 3.0) * TA(f[idx + s] - f[idx - s]);
  acc += TA(-1.0 / 12.0) * TA(f[idx + 2 * s] - f[idx - 2 * s]);
  return acc;
}

// Periodic central first derivative (z direction).
template <int ORDER, class TA, class TD>
__device__ __forceinline__ TA dper(const TD* __restrict__ f, long idx, long s, int i, int n) {
  const long base = idx - (long)i * s;
  auto at = [&](int m) {
    int q = i + m;
    q = q < 0 ? q + n : (q >= n ? q - n : q);
    return f[base + (long)q * s];
  };
  if (ORDER == 6) {
    TA acc = TA(0.75) * TA(at(1) - at(-1));
    acc += TA(-0.15) * TA(at(2) - at(-2));
    acc += TA(1.0 / 60.0) * TA(at(3) - at(-3));
    return acc;
  }
  TA acc = TA(2.0 / 3.0) * TA(at(1) - at(-1));
  acc += TA(-1.0 / 12.0) * TA(at(2) - at(-2));
  return acc;
}

// The 8 XCDs of the chip take workgroups round-robin (workgroup b goes to XCD b mod 8).
// Stencil kernels remap b so that each XCD sweeps one contiguous band of grid rows:
// the y (and z) neighbours a tile reads are then mostly in that XCD's own L2.
__device__ __forceinline__ long xcd_block() {
  const long b = blockIdx.x, nb = gridDim.x;
  const long per = nb >> 3;
  if (b >= (per << 3)) return b;
  return (b & 7) * per + (b >> 3);
}

// Periodic index of q in [-n, 3n) on a line of n points (a 3-D tile's z halo reaches up
// to 11 planes past the last tile origin, which is more than one period when nz = 9)
__device__ __forceinline__ int wrap_per(int q, int n) {
  q = q < 0 ? q + n : q;
  q = q >= n ? q - n : q;
  return q >= n ? q - n : q;
}

// Values a kernel touches once and no other block re-reads (the point's own state,
// fluxes and updates) are loaded and stored with the nontemporal hint, so that they do
// not displace from L2 the stencil neighbours that nearby blocks read again (measured on
// the 512 x 256 x 128 jet: flux -4 %, 3-D divergence -3.5 %, same bits; on the 2-D SBLI the flux
// -3 % from the loads alone).
template <class T>
__device__ __forceinline__ T ld_once(const T* p) { return __builtin_nontemporal_load(p); }
template <class T>
__device__ __forceinline__ void st_once(T v, T* p) { __builtin_nontemporal_store(v, p); }

// Branch-free form of the same first-derivative operators: D f = sum_m a_m (f[p_m] - f[q_m])
// over at most four pairs.  The pairs depend only on the position along the line, so
// one Sten serves every field at a point and all field loads can be issued together.
//   interior (6th): (i+1,i-1, 3/4), (i+2,i-2, -3/20), (i+3,i-3, 1/60)
//   interior (4th) and points 2, n-3 of the 6th-order operator: (i+1,i-1, 2/3), (i+2,i-2, -1/12)
//   point 0: (m, 0, b0_m) for m = 1..4; point 1: (m, 1, b1_m) for m = 0, 2, 3, 4
//   (the closure weights sum to zero, so they act on differences to the point itself);
//   points n-1, n-2: mirror images with the sign flipped.
struct Sten {
  long p[4], q[4];
  double a[4];
};

template <int ORDER>
__device__ __forceinline__ Sten make_sten(long idx, long s, int i, int n) {
  // row class: 0 = central 6th order, 1 = central 4th order, 2 = boundary point,
  // 3 = first point off the boundary.  Offsets and weights are formed with selects
  // (no per-class branches, so the stencil lives in registers, not private memory).
  const bool c6 = ORDER == 6 && i >= 3 && i <= n - 4;
  const bool c4 = (ORDER == 4 && i >= 2 && i <= n - 3) ||
                  (ORDER == 6 && (i == 2 || i == n - 3));
  const int cls = c6 ? 0 : (c4 ? 1 : ((i == 0 || i == n - 1) ? 2 : 3));
  const bool lo = 2 * i < n;                  // closure at the low end of the line
  const long sg = (cls >= 2 && !lo) ? -s : s;
  const double f = (cls >= 2 && !lo) ? -1.0 : 1.0;
  const bool cen = cls < 2;
  Sten t;
  t.p[0] = cls == 3 ? idx - sg : idx + sg;
  t.p[1] = cls == 3 ? idx + sg : idx + 2 * sg;
  t.p[2] = cls == 3 ? idx + 2 * sg : (cls == 1 ? idx : idx + 3 * sg);
  t.p[3] = cls == 3 ? idx + 3 * sg : (cls == 2 ? idx + 4 * sg : idx);
  t.q[0] = cen ? idx - s : idx;
  t.q[1] = cen ? idx - 2 * s : idx;
  t.q[2] = cls == 0 ? idx - 3 * s : idx;
  t.q[3] = idx;
  t.a[0] = cls == 0 ? 0.75 : (cls == 1 ? 2.0 / 3.0 : (cls == 2 ? 4.0 * f : -0.25 * f));
  t.a[1] = cls == 0 ? -0.15 : (cls == 1 ? -1.0 / 12.0 : (cls == 2 ? -3.0 * f : 1.5 * f));
  t.a[2] = cls == 0 ? 1.0 / 60.0 : (cls == 1 ? 0.0 : (cls == 2 ? (4.0 / 3.0) * f : -0.5 * f));
  t.a[3] = cen ? 0.0 : (cls == 2 ? -0.25 * f : (1.0 / 12.0) * f);
  return t;
}

template <int ORDER>
__device__ __forceinline__ Sten make_sten_per(long idx, long s, int i, int n) {
  Sten t;
  const long base = idx - (long)i * s;
  auto at = [&](int m) {
    int q = i + m;
    q = q < 0 ? q + n : (q >= n ? q - n : q);
    return base + (long)q * s;
  };
  t.p[3] = idx; t.q[3] = idx; t.a[3] = 0.0;
  if (ORDER == 6) {
    t.p[0] = at(1); t.q[0] = at(-1); t.a[0] = 0.75;
    t.p[1] = at(2); t.q[1] = at(-2); t.a[1] = -0.15;
    t.p[2] = at(3); t.q[2] = at(-3); t.a[2] = 1.0 / 60.0;
  } else {
    t.p[0] = at(1); t.q[0] = at(-1); t.a[0] = 2.0 / 3.0;
    t.p[1] = at(2); t.q[1] = at(-2); t.a[1] = -1.0 / 12.0;
    t.p[2] = idx; t.q[2] = idx; t.a[2] = 0.0;
  }
  return t;
}

// differences in the storage type TD, weighted sum in the arithmetic type TA; NP = number
// of pairs used (interior points of the 6th/4th-order operators need 3/2, closures 4)
template <class TA, int NP = 4, class TD>
__device__ __forceinline__ TA sten_apply(const Sten& t, const TD* __restrict__ f) {
  TD d[NP];
#pragma unroll
  for (int m = 0; m < NP; ++m) d[m] = f[t.p[m]] - f[t.q[m]];
  TA acc = TA(t.a[0]) * TA(d[0]);
#pragma unroll
  for (int m = 1; m < NP; ++m) acc += TA(t.a[m]) * TA(d[m]);
  return acc;
}

// true when the point is interior to every non-periodic line (central stencil only)
template <int ORDER>
__device__ __forceinline__ bool interior_point(const Dev& d, int i, int j) {
  const int h = ORDER == 6 ? 3 : 2;
  return i >= h && i <= d.nx - 1 - h && j >= h && j <= d.ny - 1 - h;
}

struct Pt {
  long idx;
  int i, j, k;
};

// Stencil kernels run on a grid of gx * ny * nz blocks of 128 threads, block = 128
// consecutive x points of one grid row (gx = ceil(nx / 128)); blockIdx.y, when used,
// selects a field component.  The XCD-aware block number is decomposed into
// (x segment, row j, plane k) with 32-bit arithmetic.
constexpr int TX = 128;

__device__ __forceinline__ bool grid_point(const Dev& d, Pt& p) {
  const unsigned b = (unsigned)blockIdx.x, nb = gridDim.x;
  const unsigned per = nb >> 3;
  const unsigned L = b >= (per << 3) ? b : (b & 7u) * per + (b >> 3);
  const unsigned gx = (unsigned)d.gx;
  const unsigned r = L / gx;
  p.i = (int)((L - r * gx) * TX + threadIdx.x);
  p.j = (int)(r % (unsigned)d.ny);
  p.k = (int)(r / (unsigned)d.ny);
  p.idx = ((long)p.k * d.ny + p.j) * d.nx + p.i;
  return p.i < d.nx;
}

// Same grid with the plane index k varying fastest (then the x segment, then the row
// j): the blocks an XCD runs back to back hold z-neighbours, which its L2 then serves.
// For kernels whose only stencil runs along z.
__device__ __forceinline__ bool grid_point_zfast(const Dev& d, Pt& p) {
  const unsigned b = (unsigned)blockIdx.x, nb = gridDim.x;
  const unsigned per = nb >> 3;
  const unsigned L = b >= (per << 3) ? b : (b & 7u) * per + (b >> 3);
  const unsigned nz = (unsigned)d.nz, gx = (unsigned)d.gx;
  const unsigned r = L / nz;
  p.k = (int)(L - r * nz);
  const unsigned jr = r / gx;
  p.i = (int)((r - jr * gx) * TX + threadIdx.x);
  p.j = (int)jr;
  p.idx = ((long)p.k * d.ny + p.j) * d.nx + p.i;
  return p.i < d.nx;
}

// 2-D stencil tiles staged through LDS: a block of 256 threads owns TTX x TTY points
// and loads its source planes with a halo of 4 on each side (TW x TH values per plane;
// 4 = the reach of the one-sided closures from an end point) in one pass of
// independent loads before a single barrier; halo values outside the domain are
// clamped copies that the closures never use.  32 x 8 measured faster than 64 x 4 and
// 16 x 16 (less halo per point in 2-D; in 3-D a narrower x tile keeps the y-neighbour
// rows of a tile column within one XCD's L2).
constexpr int TTX = 32, TTY = 8, THALO = 4;
constexpr int TW = TTX + 2 * THALO, TH = TTY + 2 * THALO, TILE_E = TW * TH;
constexpr int FXE = TTY * TW, FYE = TH * TTX;   // flux tiles: x halo only, y halo only
constexpr int KCH = 4;                          // flux components staged per LDS pass
// components per pass of the divergence kernel (3-D: 9 = 3 x 3, no idle pass)
constexpr int div_chunk(int nd) { return nd == 3 ? 3 : KCH; }

// Stage TOTAL values into LDS: element e comes from src_of(e).  Every thread first issues
// all of its global loads (held in registers), then writes them, so the loads of a
// thread are in flight together instead of one round trip per element.
template <int TOTAL, int NTHREADS, class T, class SrcOf>
__device__ __forceinline__ void stage_tile(T* __restrict__ dst, SrcOf src_of,
                                           int tid = threadIdx.x) {
  constexpr int PER = (TOTAL + NTHREADS - 1) / NTHREADS;
  T v[PER];
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int e = tid + q * NTHREADS;
    v[q] = (e < TOTAL) ? src_of(e) : 0.0;
  }
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int e = tid + q * NTHREADS;
    if (e < TOTAL) dst[e] = v[q];
  }
}

__device__ __forceinline__ void tile_origin(const Dev& d, int& i0, int& j0,
                                            unsigned b = blockIdx.x, unsigned nb = gridDim.x) {
  const unsigned per = nb >> 3;
  const unsigned L = b >= (per << 3) ? b : (b & 7u) * per + (b >> 3);
  const unsigned tgx = (unsigned)d.tgx;
  const unsigned by = L / tgx;
  i0 = (int)(L - by * tgx) * TTX;
  j0 = (int)by * TTY;
}

// 3-D tiles lie in the (x, z) plane, TTX x TTY points with a halo of 4 (z periodic),
// one grid row j per block.  Consecutive blocks (one XCD's range) walk the z tiles of a
// row, then the next row: the z halo a tile stages was staged by the block before it.
__device__ __forceinline__ void tile_origin3(const Dev& d, int& i0, int& j, int& k0,
                                             unsigned b = blockIdx.x, unsigned nb = gridDim.x) {
  const unsigned per = nb >> 3;
  const unsigned L = b >= (per << 3) ? b : (b & 7u) * per + (b >> 3);
  const unsigned ny = (unsigned)d.ny, tgz = (unsigned)d.tgz;
  const unsigned t = L / tgz;
  k0 = (int)(L - t * tgz) * TTY;
  const unsigned xt = t / ny;
  j = (int)(t - xt * ny);
  i0 = (int)xt * TTX;
}

// central first-derivative stencil (periodic direction staged with its halo)
template <int ORDER>
__device__ __forceinline__ Sten make_sten_central(long idx, long s) {
  Sten t;
  t.p[0] = idx + s; t.q[0] = idx - s;
  t.p[1] = idx + 2 * s; t.q[1] = idx - 2 * s;
  t.p[2] = ORDER == 6 ? idx + 3 * s : idx; t.q[2] = ORDER == 6 ? idx - 3 * s : idx;
  t.p[3] = idx; t.q[3] = idx;
  t.a[0] = ORDER == 6 ? 0.75 : 2.0 / 3.0;
  t.a[1] = ORDER == 6 ? -0.15 : -1.0 / 12.0;
  t.a[2] = ORDER == 6 ? 1.0 / 60.0 : 0.0;
  t.a[3] = 0.0;
  return t;
}

__device__ __forceinline__ Pt point_of(const Dev& d, long idx) {
  Pt p;
  p.idx = idx;
  p.i = (int)(idx % d.nx);
  long r = idx / d.nx;
  p.j = (int)(r % d.ny);
  p.k = (int)(r / d.ny);
  return p;
}

// physical derivative of plane f along direction dir at point p
template <int ORDER, class TA, class TD>
__device__ __forceinline__ TA dphys(const Dev& d, const TD* __restrict__ f, const Pt& p, int dir) {
  if (dir == 0) return dline<ORDER, TA, TD>(f, p.idx, 1, p.i, d.nx) * TA(d.mx[p.i]);
  if (dir == 1) return dline<ORDER, TA, TD>(f, p.idx, d.nx, p.j, d.ny) * TA(d.my[p.j]);
  return dper<ORDER, TA, TD>(f, p.idx, (long)d.nx * d.ny, p.k, d.nz) * TA(d.mz[p.k]);
}

// Device counters: NCOUNT kinds, each spread over CSLOTS addresses chosen by the block
// number (the host sums the slots).  A counter that many wavefronts hit in one launch
// (negative trace densities after many stages, say) would otherwise serialise the
// whole launch on one address's device-scope atomics.
constexpr int NCOUNT = 8, CSLOTS = 256;
__device__ __forceinline__ unsigned long long* cslot(unsigned long long* c, int kind) {
  return c + kind * CSLOTS + (blockIdx.x & (CSLOTS - 1));
}

__device__ __forceinline__ void count(const Dev& d, int status) {
  if (status == 1) atomicAdd(cslot(d.counters, 0), 1ull);
  if (status == 2) atomicAdd(cslot(d.counters, 1), 1ull);
}

// Count the lanes of the wavefront for which pred holds with one atomic (the first
// active lane adds the population count of the ballot).
__device__ __forceinline__ void wave_count(unsigned long long* c, int kind, bool pred) {
  const unsigned long long m = __ballot(pred);
  if (m == 0ull) return;
  const unsigned long long act = __ballot(1);
  if ((int)__lane_id() == __ffsll((long long)act) - 1)
    atomicAdd(cslot(c, kind), (unsigned long long)__popcll(m));
}

// Finite state of positive density (else the point is counted as non-finite)
__device__ __forceinline__ bool finite_state(const double* v, int n, double rho) {
  bool ok = rho > 0.0 && isfinite(rho);
#pragma unroll 9
  for (int k = 0; k < n; ++k) ok = ok && isfinite(v[k]);
  return ok;
}

// Temperature above which the mixed form keeps the Arrhenius exponentials in FP64.
constexpr double T_HI_MIXED = 2000.0;

// ------------------------------------------------------------------ k_prim
// Mole fractions and pressure of 5-species air from the partial densities, in the one
// order of operations the pointwise pass and the flux share.  In 2-D the flux forms its
// tile's X_s and its point's p itself, bit-identical to the pointwise pass, which then
// stores neither (the 3-D flux reads the y neighbours' X_s from the stored planes).
// rho = sum rho_s, Y_s = rho_s / rho, X_s = (Y_s/M_s) / sum(Y_r/M_r), p = rho T R_mix
// p_fac (T nondimensional).
__device__ __forceinline__ void air5_mole_fractions(const double* rs, double* X) {
  double rho = 0.0;
#pragma unroll
  for (int s = 0; s < NS; ++s) rho += rs[s];
  const double irho = 1.0 / rho;
  double n = 0.0;
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    X[s] = (rs[s] * irho) * (1.0 / molar_mass(s));
    n += X[s];
  }
  const double in = 1.0 / n;
#pragma unroll
  for (int s = 0; s < NS; ++s) X[s] = X[s] * in;
}
__device__ __forceinline__ double air5_pressure(const Dev& d, const double* rs, double T) {
  double rho = 0.0;
#pragma unroll
  for (int s = 0; s < NS; ++s) rho += rs[s];
  const double irho = 1.0 / rho;
  double Y[NS];
#pragma unroll
  for (int s = 0; s < NS; ++s) Y[s] = rs[s] * irho;
  return rho * T * mixture_R(Y) * d.p_fac;
}

// Wd planes (double): [u, v, (w), T, X_1..X_5 (air5), p]   -- differentiated or convective
// Wp planes (RT):     [mu, kappa, D_1..D_5, wdot_1..wdot_5, h_1..h_5, (c)] (air5),
//                     [mu, (c)] (CPG)

// Pointwise thermochemistry of one 5-species point from its conserved values (partial
// densities rs, momentum m, total energy rhoE; nondimensional): energy inversion
// (warm start from the stored temperature, else from T_start > 0, else cold), pressure,
// mole fractions, transport (plain, or, when net is set, from the surrogate's outputs
// ys = (ln T, ln mu, ln kappa, ln(rho D_s)) in SI), production rates, species
// enthalpies and, with artificial diffusivity, the sound speed.
template <int ND, class RT>
__device__ __forceinline__ void prim_air5(const Dev& d, double* __restrict__ Wd,
                                          RT* __restrict__ Wp, long idx, const double* rs,
                                          const double* mom, double rhoE, bool net,
                                          const float (&ys)[MLP_NOUT]) {
  const long N = d.N;
  double Y[NS];
  double rho = 0.0;
#pragma unroll
  for (int s = 0; s < NS; ++s) rho += rs[s];
  const double irho = 1.0 / rho;
#pragma unroll
  for (int s = 0; s < NS; ++s) Y[s] = rs[s] * irho;
  double u[3] = {0.0, 0.0, 0.0};
  double ke = 0.0;
#pragma unroll
  for (int a = 0; a < ND; ++a) {
    u[a] = mom[a] * irho;
    ke += u[a] * u[a];
  }
  const double e = rhoE * irho - 0.5 * ke;
  const double c2 = d.c_inf * d.c_inf;
  int status, iters;
  const double Tguess = d.warm ? Wd[ND * N + idx] * d.T_ref : (net ? (double)__expf(ys[0]) : 0.0);
  SpeciesThermo st;   // species state at the last Newton iterate (within rtol of Tk)
  const double Tk = temperature_from_energy(e * c2, Y, d.newton_rtol, d.newton_max, &status,
                                            &iters, Tguess, &st);
  if (status) {
    count(d, status);
    species_e_cv(Tk, st);
  }
  const double T = Tk * d.iT_ref;
  const double Rmix = mixture_R(Y);
  const double p = air5_pressure(d, rs, T);
  const double p_d = p * d.rho_inf * c2;
  double X[NS];
  air5_mole_fractions(rs, X);
  if (net) {
    // the network's logarithms carry ~1e-4 relative error: FP32 exponentials suffice
    Wp[d.w_mu * N + idx] = RT(__expf(ys[1]) * (float)d.imu_inf);
    Wp[d.w_kap * N + idx] = RT(__expf(ys[2]) * (float)d.ikappa_inf);
    const float iDr = (float)(d.iDscale / (rho * d.rho_inf));
#pragma unroll
    for (int s = 0; s < NS; ++s) Wp[(d.w_D + s) * N + idx] = RT(__expf(ys[3 + s]) * iDr);
  } else {
    Transport<RT> tr;
    mixture_transport<RT>(Tk, p_d, X, st.cv, tr);
    Wp[d.w_mu * N + idx] = tr.mu * RT(d.imu_inf);
    Wp[d.w_kap * N + idx] = tr.kappa * RT(d.ikappa_inf);
    const RT iDscale = RT(d.iDscale);
#pragma unroll
    for (int s = 0; s < NS; ++s) Wp[(d.w_D + s) * N + idx] = tr.D[s] * iDscale;
    if (d.sm) {
      // nondimensional 1/D_sr = (1/D_sr,SI) c_inf L_ref
      const RT Dscale = RT(d.c_inf * d.L_ref);
#pragma unroll
      for (int q = 0; q < 10; ++q) Wp[(d.w_iD + q) * N + idx] = tr.iD[q] * Dscale;
    }
  }
  double rsd[NS];
  RT wd[NS];
#pragma unroll
  for (int s = 0; s < NS; ++s) rsd[s] = rs[s] * d.rho_inf;
  production_rates<RT>(rsd, Tk, st.em1, wd, T_HI_MIXED);
#pragma unroll
  for (int a = 0; a < ND; ++a) Wd[a * N + idx] = u[a];
  Wd[ND * N + idx] = T;
  if (ND == 3 || d.compact) {
    // the 3-D flux and the compact line solves read X_s and p from planes
#pragma unroll
    for (int s = 0; s < NS; ++s) Wd[(ND + 1 + s) * N + idx] = X[s];
    Wd[d.w_p * N + idx] = p;
  }
#pragma unroll
  for (int s = 0; s < NS; ++s) Wp[(d.w_wdot + s) * N + idx] = RT(double(wd[s]) * d.wscale);
  if (d.ad_on) {
    double cv = 0.0;
#pragma unroll
    for (int s = 0; s < NS; ++s) cv += Y[s] * st.cv[s];
    const double gf = (cv + Rmix) / cv;
    Wp[d.w_c * N + idx] = RT(sqrt(gf * Rmix * Tk) * d.ic_inf);
    // the pointwise sources of the artificial diffusivity: e and Y_s
    RT* Aad = static_cast<RT*>(d.ad);
    Aad[2 * N + idx] = RT(e);
#pragma unroll
    for (int s = 0; s < NS; ++s) Aad[(3 + s) * N + idx] = RT(Y[s]);
  }
}

// Plain form, or (SUR) the surrogate form reading the network's outputs ys[8][N]
// (NaN in ys[0]: outside the hull, plain transport, counted).
template <int GAS, int ND, class RT, bool SUR = false>
__global__ __launch_bounds__(128) void k_prim(Dev d, const double* __restrict__ Q,
                                              double* __restrict__ Wd, RT* __restrict__ Wp,
                                              const float* __restrict__ ysin) {
  // Without artificial diffusivity each XCD takes one contiguous band of points, the band
  // its stencil blocks of the previous and next passes cover (their planes may still sit
  // in its L2; flat plate -3 %).  With it the AD passes that follow walk other orders and
  // the plain order measured better.
  const long blk = d.ad_on ? (long)blockIdx.x : xcd_block();
  const long idx = blk * blockDim.x + threadIdx.x;
  if (idx >= d.N) return;
  const long N = d.N;
  if (GAS != AIR5) {
    const double rho = Q[idx];
    {
      double qv[5];
#pragma unroll
      for (int k = 0; k < ND + 2; ++k) qv[k] = Q[(long)k * N + idx];
      wave_count(d.counters, 3, !finite_state(qv, ND + 2, rho));
      wave_count(d.counters, 4, rho < 0.0);
    }
    double u[3] = {0.0, 0.0, 0.0};
    double ke = 0.0;
#pragma unroll
    for (int a = 0; a < ND; ++a) {
      u[a] = Q[(1 + a) * N + idx] / rho;
      ke += u[a] * u[a];
    }
    const double E = Q[(1 + ND) * N + idx] / rho;
    const double e = E - 0.5 * ke;
    const double g = d.gamma;
    double T = g * e;
    if (GAS == TPG) {
      int status;
      T = tpg_temperature(e, d.tpg_k0, d.tpg_th, (g - 1.0) / g, d.newton_rtol, d.newton_max,
                          &status, d.warm ? Wd[ND * N + idx] : 0.0);
      if (status) atomicAdd(cslot(d.counters, 0), 1ull);
    }
    const double p = rho * (g - 1.0) * T / g;
    const RT mu = sutherland<RT>(RT(T * d.T_ref)) / RT(d.mu_inf);
#pragma unroll
    for (int a = 0; a < ND; ++a) Wd[a * N + idx] = u[a];
    Wd[ND * N + idx] = T;
    Wd[d.w_p * N + idx] = p;
    Wp[d.w_mu * N + idx] = mu;
    if (GAS == TPG) Wp[d.w_kap * N + idx] = RT(keyes(T * d.T_ref) * d.ikappa_inf);
    if (d.ad_on) {
      // sound speed with gamma(T) = c_p / c_v = 1 + R / c_v(T) for the thermally perfect gas
      double gT = g;
      if (GAS == TPG) {
        const double a = (g - 1.0) / g;
        gT = 1.0 + a / (d.tpg_k0 * (1.0 + a * tpg_vib(d.tpg_th / T)) - a);
      }
      Wp[d.w_c * N + idx] = RT(sqrt(gT * p / rho));
      static_cast<RT*>(d.ad)[2 * N + idx] = RT(e);
    }
    return;
  }
  double rs[NS], mom[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int s = 0; s < NS; ++s) rs[s] = Q[s * N + idx];
#pragma unroll
  for (int a = 0; a < ND; ++a) mom[a] = Q[(NS + a) * N + idx];
  {
    double qv[NS + 4], rho = 0.0;
    bool neg = false;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      qv[s] = rs[s];
      rho += rs[s];
      neg = neg || rs[s] < 0.0;
    }
#pragma unroll
    for (int a = 0; a < ND; ++a) qv[NS + a] = mom[a];
    qv[NS + ND] = Q[(NS + ND) * N + idx];
    wave_count(d.counters, 3, !finite_state(qv, NS + ND + 1, rho));
    wave_count(d.counters, 4, neg);
  }
  float ys[MLP_NOUT] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  bool net = false;
  if (SUR) {
#pragma unroll
    for (int o = 0; o < MLP_NOUT; ++o) ys[o] = ysin[o * N + idx];
    net = !isnan(ys[0]);
    if (!net) atomicAdd(cslot(d.counters, 2), 1ull);
  }
  prim_air5<ND, RT>(d, Wd, Wp, idx, rs, mom, Q[(NS + ND) * N + idx], net, ys);
}

// ------------------------------------------------------------------ artificial diffusivity
// A planes (RT): [|S|, theta, e, Y_1..Y_ns].  The pointwise pass writes e and Y_s (it
// holds them already); k_ad_src forms |S| and theta from the velocity gradient.
template <int GAS, int ND, int ORDER, class RT>
__global__ __launch_bounds__(256) void k_ad_src(Dev d, const double* __restrict__ Wd,
                                                RT* __restrict__ A) {
  // velocity planes staged like the flux's tiles: 2-D (x, y) tiles, 3-D (x, z) tiles of
  // one row with the y differences from memory
  extern __shared__ double smem[];
  const long N = d.N;
  int i0, j0, k0 = 0;
  if (ND == 2) tile_origin(d, i0, j0);
  else tile_origin3(d, i0, j0, k0);
  stage_tile<ND * TILE_E, TTX * TTY>(smem, [&](int e) {
    const int v = e / TILE_E, r = e - v * TILE_E;
    const int ly = r / TW, lx = r - ly * TW;
    const int gi = min(max(i0 + lx - THALO, 0), d.nx - 1);
    if (ND == 2) {
      const int gj = min(max(j0 + ly - THALO, 0), d.ny - 1);
      return Wd[(long)v * N + (long)gj * d.nx + gi];
    }
    int gk = k0 + ly - THALO;
    gk = wrap_per(gk, d.nz);
    return Wd[(long)v * N + ((long)gk * d.ny + j0) * d.nx + gi];
  });
  __syncthreads();
  const int tx = threadIdx.x & (TTX - 1), ty = threadIdx.x / TTX;
  Pt p;
  p.i = i0 + tx;
  p.j = ND == 2 ? j0 + ty : j0;
  p.k = ND == 2 ? 0 : k0 + ty;
  if (p.i >= d.nx || p.j >= d.ny || p.k >= d.nz) return;
  p.idx = ((long)p.k * d.ny + p.j) * d.nx + p.i;
  const long idx = p.idx;
  const long sidx = (long)(ty + THALO) * TW + tx + THALO;
  Sten sd[3];
  RT md[3];
  sd[0] = make_sten<ORDER>(sidx, 1, p.i, d.nx);
  md[0] = RT(d.mx[p.i]);
  md[1] = RT(d.my[p.j]);
  if (ND == 2) {
    sd[1] = make_sten<ORDER>(sidx, TW, p.j, d.ny);
  } else {
    sd[1] = make_sten<ORDER>(0, d.nx, p.j, d.ny);   // offsets from the point (row-uniform)
    sd[2] = make_sten_central<ORDER>(sidx, TW);
    md[2] = RT(d.mz[p.k]);
  }
  constexpr int NPI = ORDER == 6 ? 3 : 2;
  RT G[3][3];
#pragma unroll
  for (int a = 0; a < ND; ++a)
#pragma unroll
    for (int b = 0; b < ND; ++b) {
      const double* f = smem + a * TILE_E;
      RT g;
      if (b == 2) g = sten_apply<RT, NPI>(sd[2], f);
      else if (ND == 3 && b == 1) g = sten_apply<RT>(sd[1], Wd + (long)a * N + idx);
      else g = sten_apply<RT>(sd[b], f);
      G[a][b] = g * md[b];
    }
  RT s2 = RT(0);
#pragma unroll
  for (int a = 0; a < ND; ++a)
#pragma unroll
    for (int b = 0; b < ND; ++b) {
      const RT sab = RT(0.5) * (G[a][b] + G[b][a]);
      s2 += sab * sab;
    }
  RT theta = RT(0);
#pragma unroll
  for (int a = 0; a < ND; ++a) theta += G[a][a];
  A[0 * N + idx] = sqrt(s2);
  A[1 * N + idx] = theta;
}


// 9-point truncated Gaussian filter (Gaussian weights renormalised at non-periodic
// ends; x and y are filtered inside k_ad_march), here along the periodic z direction
__constant__ double c_gauss9[5] = {3565.0 / 10368.0, 3091.0 / 12960.0, 1997.0 / 25920.0,
                                   149.0 / 12960.0, 107.0 / 103680.0};

// The z filter as a march along z: a wavefront owns 64 consecutive x points of one row
// j, a segment of ZSEG planes and one AD plane, keeps the nine taps of its column in
// registers and reads each input value once (plus the 8 planes a segment starts with).
constexpr int ZSEG = 64;
template <class RT>
__global__ __launch_bounds__(64) void k_ad_filter_z(Dev d, const RT* __restrict__ in,
                                                    RT* __restrict__ out, int nxs, int nzs) {
  const int nx = d.nx, ny = d.ny, nz = d.nz;
  const long N = d.N, P = (long)nx * ny;
  const unsigned b = (unsigned)blockIdx.x, nb = gridDim.x;
  const unsigned per = nb >> 3;
  unsigned t = b >= (per << 3) ? b : (b & 7u) * per + (b >> 3);
  // block -> (x strip fastest, row, z segment, AD plane)
  const unsigned tx = t / (unsigned)nxs;
  const int xs = (int)(t - tx * (unsigned)nxs);
  const unsigned tj = tx / (unsigned)ny;
  const int j = (int)(tx - tj * (unsigned)ny);
  const unsigned tz = tj / (unsigned)nzs;
  const int zs = (int)(tj - tz * (unsigned)nzs);
  const int v = (int)tz;
  const int i = xs * 64 + (int)threadIdx.x;
  if (i >= nx) return;
  const RT* f = in + (long)v * N + (long)j * nx + i;
  RT* o = out + (long)v * N + (long)j * nx + i;
  const int z0 = zs * ZSEG, z1 = min(z0 + ZSEG, nz);
  auto at = [&](int q) {
    q = wrap_per(q, nz);
    return f[(long)q * P];
  };
  RT w[9];   // planes k - 4 .. k + 4
#pragma unroll
  for (int m = 0; m < 8; ++m) w[m] = at(z0 - 4 + m);
  RT pf = at(z0 + 4);
  for (int k = z0; k < z1; ++k) {
    w[8] = pf;
    if (k + 1 < z1) pf = at(k + 5);
    RT r = RT(c_gauss9[0]) * w[4];
#pragma unroll
    for (int m = 1; m <= 4; ++m) r += RT(c_gauss9[m]) * (w[4 - m] + w[4 + m]);
    o[(long)k * P] = r;
#pragma unroll
    for (int m = 0; m < 8; ++m) w[m] = w[m + 1];
  }
}

// Fourth difference -> x filter -> y filter in one pass, as a march down y: a
// wavefront owns a strip of MW fourth-difference columns (MO = MW - 8 output columns,
// the x filter's halo of 4 on each side) and a segment of mseg output rows of one AD
// plane (and one z plane in 3-D), and walks down the rows.  Lane l keeps its column's
// five source rows (the fourth difference's y taps) and nine x-filtered rows (the y
// filter's taps) in registers and exchanges only the current row through LDS for the x
// taps: one global read per source value and about 17 LDS accesses per output.  A
// segment starts 4 rows early (the y filter's reach).  Within two points of a
// non-periodic end the fourth difference is the one centred two points in (the stencil
// never leaves the line); filter taps outside the domain carry zero weight and the
// weights are renormalised.  The z filter of 3-D grids follows as its own pass.
// Memory reads inside the march are loaded one row before their use and consumed before
// their register is refilled, every row refills whatever it did (lanes and wavefronts
// that need no value read a valid one), and the rows' spacings come from LDS: the vector
// memory counter is waited on in order, so a conditional load, a load used in its own
// row or a register moved while its load is in flight makes the wait drain every load in
// flight (measured on the 512 x 256 x 128 jet: 1.30 -> 0.85 ms with the 3-D form below).
// Segments of 24 rows in 2-D (SBLI: about six wavefronts per SIMD, all resident) and 128
// in 3-D (fewer halo rows; the grid still has 20 blocks per CU) -- measured.
constexpr int MW = 64, MO = MW - 8, MSEG2 = 24, MSEG3 = 128;
constexpr int AD_MARCH_NWZ = 4;   // z planes (wavefronts) per block of the 3-D march
constexpr int AD_MARCH_PD = 1;    // rows a wavefront's loads run ahead (more: more registers)
template <int GAS, class RT>
__global__ __launch_bounds__(MW) void k_ad_march(Dev d, const RT* __restrict__ A,
                                                RT* __restrict__ B, int nstrip, int nseg,
                                                int mseg) {
  __shared__ RT sa[MW + 4];   // source row q, columns i0 - 6 .. i0 + MW - 3
  __shared__ RT sd[MW];       // fourth differences of row q, columns i0 - 4 .. i0 + MW - 5
  __shared__ double sdly[MSEG2 + 8];
  const int nx = d.nx, ny = d.ny;
  const long N = d.N;
  const unsigned b = (unsigned)blockIdx.x, nb = gridDim.x;
  const unsigned per = nb >> 3;
  unsigned t = b >= (per << 3) ? b : (b & 7u) * per + (b >> 3);
  // block -> (strip, segment, AD plane)
  const unsigned ts = t / (unsigned)nstrip;
  const int strip = (int)(t - ts * (unsigned)nstrip);
  const unsigned tg = ts / (unsigned)nseg;
  const int seg = (int)(ts - tg * (unsigned)nseg);
  const int v = (int)tg;
  const int l = threadIdx.x;
  const int i0 = strip * MO, y0 = seg * mseg, y1 = min(y0 + mseg, ny);
  const RT* f = A + (long)v * N;
  const bool sq = v < 2;
  // the lane's fourth-difference column, the centre of its x taps, its spacing
  const int gx = min(max(i0 - 4 + l, 0), nx - 1);
  const int ic = gx < 2 ? 2 : (gx > nx - 3 ? nx - 3 : gx);
  const int jx = ic - 2 - (i0 - 6);           // first x tap in sa
  const double dlxg = d.dlx[gx];
  const RT dlx = RT(dlxg);
  const RT wxf = sq ? dlx * dlx : dlx;
  // extra source columns for the x taps of the strip's end columns (lanes 0..3; the
  // other lanes read their own column there)
  const int ex = l < 2 ? i0 - 6 + l : i0 + MW - 6 + l;   // l = 2, 3 -> i0 + MW - 4, - 3
  const int gex = l < 4 ? min(max(ex, 0), nx - 1) : gx;
  const int sex = l < 2 ? l : MW + l;                     // its slot in sa
  // x filter of output lane l (column i0 - 4 + l, lanes 4 .. MW - 5)
  RT wxs = RT(0);
  const int ocol = i0 - 4 + l;
#pragma unroll
  for (int m = -4; m <= 4; ++m) {
    const int q = ocol + m;
    wxs += (q >= 0 && q < nx) ? RT(c_gauss9[m < 0 ? -m : m]) : RT(0);
  }
  // sd holds zero for columns outside the domain: their taps then add nothing, as a
  // zero weight would, with the filter's coefficients as constants
  const bool incol = ocol >= 0 && ocol < nx;
  const bool olane = l >= 4 && l < MW - 4 && ocol < nx;
  const RT iwx = olane ? RT(1) / wxs : RT(0);
  const int xl = min(max(l, 4), MW - 5) - 4;   // first x-filter tap in sd (in range)
  const int qs = y0 - 4, qe = y1 + 3;
  for (int m = l; m <= qe - qs; m += MW) {
    const int q = qs + m;
    sdly[m] = (q >= 0 && q < ny) ? d.dly[q] : 0.0;
  }
  // the y taps: rows c - 2 .. c + 2 of the column, c = the row clamped to [2, ny - 3];
  // the first row in range sets c, and every later row q with 3 <= q <= ny - 3 advances
  // it by one, taking row q + 2 from pq (refilled with the next advancing row's)
  auto row = [&](int r, int col) { return f[(long)min(max(r, 0), ny - 1) * nx + col]; };
  const int q0 = max(qs, 0);
  const int c0 = min(max(q0, 2), ny - 3);
  const int qa = max(q0 + 1, 3);   // the first row that may advance
  RT a0 = row(c0 - 2, gx), a1 = row(c0 - 1, gx), a2 = row(c0, gx), a3 = row(c0 + 1, gx),
     a4 = row(c0 + 2, gx);
  RT pq = row(qa + 2, gx);   // row (next advancing row) + 2
  RT eq = row(q0, gex);      // the extra column's row q
  // interior y-filter weight sum (every tap inside the domain), in the filter's order
  RT wint = RT(0);
#pragma unroll
  for (int m = -4; m <= 4; ++m) wint += RT(c_gauss9[m < 0 ? -m : m]);
  const RT iwint = RT(1) / wint;
  RT xr[9];
#pragma unroll
  for (int m = 0; m < 9; ++m) xr[m] = RT(0);
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  for (int q = qs; q <= qe; ++q) {
    RT xf = RT(0);
    if (q >= 0 && q < ny) {
      if (q > q0 && q >= 3 && q <= ny - 3) {
        a0 = a1; a1 = a2; a2 = a3; a3 = a4; a4 = pq;
      }
      const int cq = min(max(q, 2), ny - 3);
      RT aq = a2;   // row q in the ring (its centre away from the ends)
      if (q != cq) {
        const int dq = q - cq;
        aq = dq < 0 ? (dq == -1 ? a1 : a0) : (dq == 1 ? a3 : a4);
      }
      sa[l + 2] = aq;
      if (l < 4) sa[sex] = eq;
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      const RT* ax = sa + jx;
      const RT qx = ax[0] - RT(4) * ax[1] + RT(6) * ax[2] - RT(4) * ax[3] + ax[4];
      const RT qy = a0 - RT(4) * a1 + RT(6) * a2 - RT(4) * a3 + a4;
      const double dlyq = sdly[q - qs];
      const RT dly = RT(dlyq);
      RT acc = RT(0);
      acc += qx * wxf;
      acc += qy * (sq ? dly * dly : dly);
      RT out = fabs(acc);
      if (GAS == AIR5 && v >= 3) {
        const RT over = RT(0.5) * (fabs(aq) - RT(1) + fabs(RT(1) - aq));
        out = RT(d.CD) * out;
        if (over != RT(0)) {
          const RT fdb = RT(sqrt(dlxg * dlyq));
          out = out + RT(d.CY) * over * fdb;
        }
      }
      sd[l] = incol ? out : RT(0);
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      RT xa = RT(0);
#pragma unroll
      for (int m = 0; m < 9; ++m) xa += RT(c_gauss9[m < 4 ? 4 - m : m - 4]) * sd[xl + m];
      xf = xa * iwx;
      // sa and sd are rewritten next row only after every lane's reads above
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    // refills, whatever the row did, into the registers just read
    pq = row(max(q + 1, qa) + 2, gx);
    eq = row(max(q + 1, q0), gex);
#pragma unroll
    for (int m = 0; m < 8; ++m) xr[m] = xr[m + 1];
    xr[8] = xf;
    const int r = q - 4;   // output row: x-filtered rows r - 4 .. r + 4 are in xr
    if (r >= y0 && r < y1) {
      RT yacc = RT(0), res;
      if (r >= 4 && r < ny - 4) {
#pragma unroll
        for (int m = -4; m <= 4; ++m) yacc += RT(c_gauss9[m < 0 ? -m : m]) * xr[m + 4];
        res = yacc * iwint;
      } else {
        RT wsum = RT(0);
#pragma unroll
        for (int m = -4; m <= 4; ++m) {
          const int qq = r + m;
          const RT w = (qq >= 0 && qq < ny) ? RT(c_gauss9[m < 0 ? -m : m]) : RT(0);
          yacc += w * xr[m + 4];
          wsum += w;
        }
        res = yacc / wsum;
      }
      if (olane) B[(long)v * N + (long)r * nx + ocol] = res;
    }
  }
}

// The same pass in 3-D with the z taps of the fourth difference exchanged in LDS: a block
// of NWZ wavefronts owns NWZ consecutive z planes of one strip, segment and AD plane
// (wavefront w: plane k0 + w, z periodic), each marching down the rows as above.  At
// every row each wavefront puts its row value into a z buffer (slot w + 2), and
// wavefronts 0..3 also put the row of the planes k0 - 2, k0 - 1, k0 + NWZ, k0 + NWZ + 1
// (slots 0, 1, NWZ + 2, NWZ + 3); after one block barrier the planes k +- 1, k +- 2 of
// every wavefront's point are in LDS, where the one-wavefront march reads them from
// memory.  The z buffer alternates between two halves by row, so one barrier per row
// suffices.  Wavefronts whose plane lies past nz (a partial last group) carry the
// periodic image of their plane and write nothing.
// Every value a wavefront reads from memory inside the march is loaded PD rows before
// its use, into one of PD rotating registers (slot = row mod PD; the rows are unrolled by
// PD and a segment starts at a multiple of PD), and the y spacings come from LDS: the
// vector memory counter is waited on in order, so a load used in its own row, or a
// register moved while its load is in flight, would drain every load in flight.
template <int GAS, class RT, int NWZ, int PD>
__global__ __launch_bounds__(MW * NWZ) void k_ad_march3(Dev d, const RT* __restrict__ A,
                                                       RT* __restrict__ B, int nstrip,
                                                       int nseg, int mseg, int nzg) {
  static_assert(NWZ >= 4, "wavefronts 0..3 load the halo planes");
  static_assert(4 % PD == 0 && MSEG3 % PD == 0, "segments start at a multiple of PD");
  __shared__ RT sa_all[NWZ][MW + 4];   // per wavefront: source row q, columns i0 - 6 ..
  __shared__ RT sd_all[NWZ][MW];       // per wavefront: fourth differences of row q
  __shared__ RT zb[2][NWZ + 4][MW];    // row q of planes k0 - 2 .. k0 + NWZ + 1
  __shared__ double sdly[MSEG3 + 8];  // the segment's y spacings (rows qs .. qe)
  const int nx = d.nx, ny = d.ny, nz = d.nz;
  const long N = d.N, P = (long)nx * ny;
  const unsigned b = (unsigned)blockIdx.x, nb = gridDim.x;
  const unsigned per = nb >> 3;
  unsigned t = b >= (per << 3) ? b : (b & 7u) * per + (b >> 3);
  // block -> (z group fastest, strip, segment, AD plane)
  const unsigned tk = t / (unsigned)nzg;
  const int zg = (int)(t - tk * (unsigned)nzg);
  t = tk;
  const unsigned ts = t / (unsigned)nstrip;
  const int strip = (int)(t - ts * (unsigned)nstrip);
  const unsigned tg = ts / (unsigned)nseg;
  const int seg = (int)(ts - tg * (unsigned)nseg);
  const int v = (int)tg;
  const int w = threadIdx.x / MW, l = threadIdx.x - w * MW;
  const int k0 = zg * NWZ;
  const bool kact = k0 + w < nz;            // this wavefront's plane is a real one
  const int k = (k0 + w) % nz;
  RT* sa = sa_all[w];
  RT* sd = sd_all[w];
  const int i0 = strip * MO, y0 = seg * mseg, y1 = min(y0 + mseg, ny);
  const long kb = (long)k * P;
  const RT* f = A + (long)v * N + kb;       // this plane
  const bool sq = v < 2;
  const int gx = min(max(i0 - 4 + l, 0), nx - 1);
  const int ic = gx < 2 ? 2 : (gx > nx - 3 ? nx - 3 : gx);
  const int jx = ic - 2 - (i0 - 6);
  const RT dlx = RT(d.dlx[gx]);
  const RT wxf = sq ? dlx * dlx : dlx;
  const int ex = l < 2 ? i0 - 6 + l : i0 + MW - 6 + l;
  // lanes 4.. read their own column in the extra-column slots (loads stay unconditional)
  const int gex = l < 4 ? min(max(ex, 0), nx - 1) : gx;
  const int sex = l < 2 ? l : MW + l;
  RT wxs = RT(0);
  const int ocol = i0 - 4 + l;
#pragma unroll
  for (int m = -4; m <= 4; ++m) {
    const int q = ocol + m;
    wxs += (q >= 0 && q < nx) ? RT(c_gauss9[m < 0 ? -m : m]) : RT(0);
  }
  const bool incol = ocol >= 0 && ocol < nx;
  const bool olane = kact && l >= 4 && l < MW - 4 && ocol < nx;
  const RT iwx = olane ? RT(1) / wxs : RT(0);
  const int xl = min(max(l, 4), MW - 5) - 4;
  // the halo plane this wavefront reads (wavefronts 0..3), periodic in z
  // (wavefronts 4.. read their own plane in the halo slots: loads stay unconditional)
  const int hk = w < 2 ? k0 - 2 + w : (w < 4 ? k0 + NWZ + (w - 2) : k0 + w);
  const RT* fh = A + (long)v * N + (long)(((hk % nz) + nz) % nz) * P;
  const int hslot = w < 2 ? w : NWZ + w;    // w = 2, 3 -> slots NWZ + 2, NWZ + 3
  const double dlxg = d.dlx[gx], dlzk = d.dlz[k];
  const RT fdz = RT(dlzk);
  const RT wzf = sq ? fdz * fdz : fdz;
  const int qs = y0 - 4, qe = y1 + 3;
  for (int m = threadIdx.x; m <= qe - qs; m += MW * NWZ) {
    const int q = qs + m;
    sdly[m] = (q >= 0 && q < ny) ? d.dly[q] : 0.0;
  }
  // the fourth difference's y taps: rows c - 2 .. c + 2 of the column, c = the row
  // clamped to [2, ny - 3]; the first row in range sets c, and every later row q with
  // 3 <= q <= ny - 3 advances it by one, taking row q + 2 from slot (q - qs) mod PD
  const int q0 = max(qs, 0);
  const int c0 = min(max(q0, 2), ny - 3);
  auto row = [&](const RT* g, int r, int col) { return g[(long)min(max(r, 0), ny - 1) * nx + col]; };
  RT a0 = row(f, c0 - 2, gx), a1 = row(f, c0 - 1, gx), a2 = row(f, c0, gx),
     a3 = row(f, c0 + 1, gx), a4 = row(f, c0 + 2, gx);
  // slot s holds, for its next consuming row, row r + 2 (pq; r the next advancing row of
  // the slot) and row r (hq, eq; r the next row of the slot in range); ra[s], rb[s]: the
  // slot's first such rows.  Every row refills its slot with the row its next consumer
  // needs (the same row again when it consumed nothing)
  const int qa = max(q0 + 1, 3);   // the first row that may advance
  int ra[PD], rb[PD];
  RT pq[PD], hq[PD], eq[PD];
#pragma unroll
  for (int s = 0; s < PD; ++s) {
    ra[s] = qa + (((s - (qa - qs)) % PD) + PD) % PD;
    rb[s] = q0 + (((s - (q0 - qs)) % PD) + PD) % PD;
    pq[s] = row(f, ra[s] + 2, gx);
    hq[s] = row(fh, rb[s], gx);
    eq[s] = row(f, rb[s], gex);
  }
  RT wint = RT(0);
#pragma unroll
  for (int m = -4; m <= 4; ++m) wint += RT(c_gauss9[m < 0 ? -m : m]);
  const RT iwint = RT(1) / wint;
  RT xr[9];
#pragma unroll
  for (int m = 0; m < 9; ++m) xr[m] = RT(0);
  __syncthreads();   // sdly
  for (int qb = qs; qb <= qe; qb += PD) {
#pragma unroll
    for (int u = 0; u < PD; ++u) {
      const int q = qb + u;   // slot u: (q - qs) mod PD == u
      const bool live = q <= qe;   // uniform (the last group may run past the segment)
      RT xf = RT(0);
      if (live && q >= 0 && q < ny) {   // uniform across the block
        if (q > q0 && q >= 3 && q <= ny - 3) {
          a0 = a1; a1 = a2; a2 = a3; a3 = a4; a4 = pq[u];
        }
        const int cq = min(max(q, 2), ny - 3);
        RT aq = a2;
        if (q != cq) {
          const int dq = q - cq;
          aq = dq < 0 ? (dq == -1 ? a1 : a0) : (dq == 1 ? a3 : a4);
        }
        RT (*z)[MW] = zb[q & 1];
        z[w + 2][l] = aq;
        if (w < 4) z[hslot][l] = hq[u];
        sa[l + 2] = aq;
        if (l < 4) sa[sex] = eq[u];
        __syncthreads();
        const RT* ax = sa + jx;
        const RT qx = ax[0] - RT(4) * ax[1] + RT(6) * ax[2] - RT(4) * ax[3] + ax[4];
        const RT qy = a0 - RT(4) * a1 + RT(6) * a2 - RT(4) * a3 + a4;
        const double dlyq = sdly[q - qs];
        const RT dly = RT(dlyq);
        RT acc = RT(0);
        acc += qx * wxf;
        acc += qy * (sq ? dly * dly : dly);
        {
          const RT qz = z[w][l] - RT(4) * z[w + 1][l] + RT(6) * aq - RT(4) * z[w + 3][l] +
                        z[w + 4][l];
          acc += qz * wzf;
        }
        RT out = fabs(acc);
        if (GAS == AIR5 && v >= 3) {
          const RT over = RT(0.5) * (fabs(aq) - RT(1) + fabs(RT(1) - aq));
          out = RT(d.CD) * out;
          if (over != RT(0)) {
            const RT fdb = RT(cbrt(dlxg * dlyq * dlzk));
            out = out + RT(d.CY) * over * fdb;
          }
        }
        sd[l] = incol ? out : RT(0);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        RT xa = RT(0);
#pragma unroll
        for (int m = 0; m < 9; ++m) xa += RT(c_gauss9[m < 4 ? 4 - m : m - 4]) * sd[xl + m];
        xf = xa * iwx;
        // sa and sd are rewritten next row only after every lane's reads above
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      }
      // the slot's refills, issued whatever the row did, into the registers just read
      pq[u] = row(f, max(q + PD, ra[u]) + 2, gx);
      hq[u] = row(fh, max(q + PD, rb[u]), gx);
      eq[u] = row(f, max(q + PD, rb[u]), gex);
#pragma unroll
      for (int m = 0; m < 8; ++m) xr[m] = xr[m + 1];
      xr[8] = xf;
      const int r = q - 4;
      if (live && r >= y0 && r < y1) {
        RT yacc = RT(0), res;
        if (r >= 4 && r < ny - 4) {
#pragma unroll
          for (int m = -4; m <= 4; ++m) yacc += RT(c_gauss9[m < 0 ? -m : m]) * xr[m + 4];
          res = yacc * iwint;
        } else {
          RT wsum = RT(0);
#pragma unroll
          for (int m = -4; m <= 4; ++m) {
            const int qq = r + m;
            const RT wgt = (qq >= 0 && qq < ny) ? RT(c_gauss9[m < 0 ? -m : m]) : RT(0);
            yacc += wgt * xr[m + 4];
            wsum += wgt;
          }
          res = yacc / wsum;
        }
        if (olane) st_once(res, &B[(long)v * N + kb + (long)r * nx + ocol]);
      }
    }
  }
}

// ------------------------------------------------------------------ k_flux
// 3-D tiles apply the z filter of the artificial-diffusivity planes in the flux kernel
// (their z halo is the filter's reach) instead of a pass of its own
constexpr bool FLUX_ZFILTER = true;
// F planes (double): F[j][k] for direction j and conserved component k.  Convective
// fluxes are formed in FP64; stresses, heat and diffusion fluxes in RT.
// CG: the gradients come from planes Gc[b][a] (direction b, source a; the compact
// scheme's line solves), one thread per point, no tile.
template <int GAS, int ND, int ORDER, bool AD, class RT, bool SM, bool CG = false,
          bool ZF = false>
__device__ __forceinline__ void flux_tile(const Dev& d, const double* __restrict__ Q,
                                          const double* __restrict__ Wd,
                                          const RT* __restrict__ Wp,
                                          const RT* __restrict__ Gad, double* __restrict__ F,
                                          const double* __restrict__ Gc = nullptr) {
  constexpr int ns = (GAS == AIR5) ? NS : 1;
  constexpr int nvar = ns + ND + 1;
  constexpr bool XQ = GAS == AIR5 && ND == 2 && !CG;   // X_s and p formed here from Q
  constexpr int NSRC = ND + 1 + (GAS == AIR5 ? NS : 0);   // u, v, (w), T, (X_s)
  // mole-fraction derivatives formed per flux direction (fewer live registers) where the
  // kernel is register bound: with artificial diffusivity and in 3-D (measured)
  // (the Stefan-Maxwell system takes every direction's gradients at once)
  constexpr bool DX_PER_DIR = (AD || ND == 3) && !(SM && GAS == AIR5);
  extern __shared__ double smem[];
  const long N = d.N;
  // ZF (3-D tiles): Gad holds the AD planes before their z filter, applied here
  constexpr int NADP = 3 + (GAS == AIR5 ? NS : 0);
  RT gz[NADP];
  Pt p;
  long sidx = 0;            // index of the point in the LDS tile
  Sten sd[3];
  if constexpr (CG) {
    const long gi = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (gi >= N) return;
    p = point_of(d, gi);
  } else {
    // 2-D: tile in (x, y); 3-D: tile in (x, z) at row j0, y differences from memory
    int i0, j0, k0 = 0;
    if (ND == 2) tile_origin(d, i0, j0);
    else tile_origin3(d, i0, j0, k0);
    // flat index of tile element r (clamped halo in x and y, periodic in z)
    auto tile_point = [&](int r) -> long {
      const int ly = r / TW, lx = r - ly * TW;
      const int gi = min(max(i0 + lx - THALO, 0), d.nx - 1);
      if (ND == 2) {
        const int gj = min(max(j0 + ly - THALO, 0), d.ny - 1);
        return (long)gj * d.nx + gi;
      }
      int gk = k0 + ly - THALO;
      gk = wrap_per(gk, d.nz);
      return ((long)gk * d.ny + j0) * d.nx + gi;
    };
    if constexpr (ND == 3 && AD && ZF) {
      // the z filter of the artificial-diffusivity planes (Gad: the planes before it),
      // with the z halo of the tile (the filter's reach) staged in the LDS the source tile
      // uses next; the same taps and order as k_ad_filter_z
      constexpr int ZE = TH * TTX;
      stage_tile<NADP * ZE, TTX * TTY>(smem, [&](int e) {
        const int v = e / ZE, r = e - v * ZE;
        const int ly = r / TTX, lx = r - ly * TTX;
        const int gi = min(i0 + lx, d.nx - 1);
        int gk = k0 + ly - THALO;
        gk = wrap_per(gk, d.nz);
        return double(Gad[(long)v * N + ((long)gk * d.ny + j0) * d.nx + gi]);
      });
      __syncthreads();
      const int tx = threadIdx.x & (TTX - 1), ty = threadIdx.x / TTX;
#pragma unroll 1   // unrolled, the flux's register allocation grew by 124 VGPRs
      for (int v = 0; v < NADP; ++v) {
        const double* c = smem + v * ZE + ty * TTX + tx;   // rows k - 4 .. k + 4
        RT r = RT(c_gauss9[0]) * RT(c[4 * TTX]);
#pragma unroll
        for (int m = 1; m <= 4; ++m)
          r += RT(c_gauss9[m]) * (RT(c[(4 - m) * TTX]) + RT(c[(4 + m) * TTX]));
        gz[v] = r;
      }
      __syncthreads();
    }
    // u, v, (w), T (and in 3-D X_s) from the pointwise pass's planes
    stage_tile<(XQ ? ND + 1 : NSRC) * TILE_E, TTX * TTY>(smem, [&](int e) {
      const int v = e / TILE_E;
      return Wd[(long)v * N + tile_point(e - v * TILE_E)];
    });
    if (XQ) {
      // X_s formed here from the partial densities (all loads first, then the planes)
      constexpr int PER = (TILE_E + TTX * TTY - 1) / (TTX * TTY);
      double rsv[PER][NS];
#pragma unroll
      for (int q = 0; q < PER; ++q) {
        const int e = threadIdx.x + q * TTX * TTY;
        const long g = tile_point(e < TILE_E ? e : 0);
#pragma unroll
        for (int s = 0; s < NS; ++s) rsv[q][s] = Q[(long)s * N + g];
      }
#pragma unroll
      for (int q = 0; q < PER; ++q) {
        const int e = threadIdx.x + q * TTX * TTY;
        if (e >= TILE_E) continue;
        double X[NS];
        air5_mole_fractions(rsv[q], X);
#pragma unroll
        for (int s = 0; s < NS; ++s) smem[(ND + 1 + s) * TILE_E + e] = X[s];
      }
    }
    __syncthreads();
    const int tx = threadIdx.x & (TTX - 1), ty = threadIdx.x / TTX;
    p.i = i0 + tx;
    p.j = ND == 2 ? j0 + ty : j0;
    p.k = ND == 2 ? 0 : k0 + ty;
    if (p.i >= d.nx || p.j >= d.ny || p.k >= d.nz) return;
    p.idx = ((long)p.k * d.ny + p.j) * d.nx + p.i;
    sidx = (long)(ty + THALO) * TW + tx + THALO;
    sd[0] = make_sten<ORDER>(sidx, 1, p.i, d.nx);
    if (ND == 2) {
      sd[1] = make_sten<ORDER>(sidx, TW, p.j, d.ny);
    } else {
      sd[1] = make_sten<ORDER>(0, d.nx, p.j, d.ny);   // offsets from the point (row-uniform)
      sd[2] = make_sten_central<ORDER>(sidx, TW);
    }
  }
  const long idx = p.idx;
  RT md[3];
  md[0] = RT(d.mx[p.i]);
  md[1] = RT(d.my[p.j]);
  if (ND == 3) md[2] = RT(d.mz[p.k]);
  constexpr int NPI = ORDER == 6 ? 3 : 2;
  // derivative of source plane a along direction b (z is periodic: central pairs only)
  auto deriv = [&](int a, int b) -> RT {
    if constexpr (CG) return RT(ld_once(&Gc[((long)b * NSRC + a) * N + idx]));
    if (ND == 3 && b == 1) return sten_apply<RT>(sd[1], Wd + (long)a * N + idx) * md[1];
    const double* f = smem + a * TILE_E;
    if (b == 2) return sten_apply<RT, NPI>(sd[b], f) * md[b];
    return sten_apply<RT>(sd[b], f) * md[b];
  };
  RT G[3][3], dT[3];
#pragma unroll
  for (int a = 0; a < ND; ++a)
#pragma unroll
    for (int b = 0; b < ND; ++b) G[a][b] = deriv(a, b);
#pragma unroll
  for (int b = 0; b < ND; ++b) dT[b] = deriv(ND, b);
  double u[3];
#pragma unroll
  for (int a = 0; a < ND; ++a) u[a] = Wd[a * N + idx];
  const RT mu = ld_once(&Wp[d.w_mu * N + idx]);
  double rho, rs[NS], pr;
  RT Y[NS];
  if (GAS != AIR5) {
    rho = Q[idx];
    pr = Wd[d.w_p * N + idx];
  } else {
    rho = 0.0;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      rs[s] = ld_once(&Q[s * N + idx]);
      rho += rs[s];
    }
#pragma unroll
    for (int s = 0; s < NS; ++s) Y[s] = RT(rs[s] / rho);
    pr = XQ ? air5_pressure(d, rs, Wd[ND * N + idx]) : ld_once(&Wd[d.w_p * N + idx]);
  }
  RT theta = RT(0);
#pragma unroll
  for (int a = 0; a < ND; ++a) theta += G[a][a];
  const RT kap = (GAS == CPG) ? mu : ld_once(&Wp[d.w_kap * N + idx]);
  RT mu_eff = mu / RT(d.Re);
  RT kap_eff = kap / RT(d.Re * d.Pr);
  RT beta = RT(0), cs = RT(0);
  const RT rho_r = RT(rho);
  if (AD) {
    const RT T = RT(Wd[ND * N + idx]);
    cs = ld_once(&Wp[d.w_c * N + idx]);
    RT w2;
    if (ND == 2) {
      w2 = (G[1][0] - G[0][1]) * (G[1][0] - G[0][1]);
    } else {
      w2 = (G[2][1] - G[1][2]) * (G[2][1] - G[1][2]) + (G[0][2] - G[2][0]) * (G[0][2] - G[2][0]) +
           (G[1][0] - G[0][1]) * (G[1][0] - G[0][1]);
    }
    const RT fsw = theta < RT(0) ? theta * theta / (theta * theta + w2 + RT(1e-32)) : RT(0);
    auto gad = [&](int v) -> RT { return ZF ? gz[v] : Gad[v * N + idx]; };
    mu_eff = mu_eff + RT(d.Cmu) * rho_r * gad(0);
    beta = RT(d.Cbeta) * rho_r * fsw * gad(1);
    kap_eff = kap_eff + RT(d.Ckap) * rho_r * cs / T * gad(2);
  }
  const double rhoE = ld_once(&Q[(ns + ND) * N + idx]);
  // species diffusion (Eq. 18 read with grad X_s)
  RT a_s[NS], h[NS];
  RT dX[NS][3];
  if (GAS == AIR5) {
    RT nsum = RT(0);
#pragma unroll
    for (int s = 0; s < NS; ++s) nsum += Y[s] / RT(molar_mass(s));
    const RT Mbar = RT(1) / nsum;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      RT Ds = SM ? RT(0) : ld_once(&Wp[(d.w_D + s) * N + idx]);
      if (AD) Ds = Ds + cs * (ZF ? gz[3 + s] : Gad[(3 + s) * N + idx]);
      a_s[s] = rho_r * (RT(molar_mass(s)) / Mbar) * Ds;
    }
    if (!DX_PER_DIR) {
#pragma unroll
      for (int s = 0; s < NS; ++s)
#pragma unroll
        for (int b = 0; b < ND; ++b) dX[s][b] = deriv(ND + 1 + s, b);
    }
    // species enthalpies h_s = e_s + R_s T (nondimensional) at the point's temperature,
    // for the diffusive heat flux (formed here rather than stored by the pointwise pass)
    {
      const double Tk = double(Wd[ND * N + idx]) * d.T_ref;
      SpeciesThermo sth;
      species_e_cv(Tk, sth);
#pragma unroll
      for (int s = 0; s < NS; ++s) h[s] = RT((sth.e[s] + gas_const(s) * Tk) * d.ic2);
    }
  }
  // Stefan-Maxwell diffusion (Eq. 17 with the driving forces of Eq. 16), in the molar
  // fluxes j_s = J_s / M_s: sum_{i != s} (X_s j_i - X_i j_s) / D_si = (rho / Mbar) dX_s,
  // i.e. C j = (rho / Mbar) grad X with C_si = X_s / D_si and C_ss = -sum_{i != s}
  // X_i / D_si.  The columns of C sum to zero; the mass constraint sum_s M_s j_s = 0
  // (Eq. 20) closes the system, added to every row: (C + alpha 1 m^T) j = (rho / Mbar)
  // grad X with m_s = M_s / Mbar and alpha the mean |C_ss| (the added term vanishes on
  // the solution).  The mole fractions enter unclipped.  The five-by-five system is
  // solved for every direction at once by Gaussian elimination with partial pivoting
  // (the row exchanges as selects, so that the matrix stays in registers); then
  // J_s = M_s j_s.  Artificial diffusivities, if any, add a flux of the form of Eq. (18)
  // with their coefficients alone (a_s below).
  constexpr bool sm = SM && GAS == AIR5;
  RT Jsm[NS][3];
  if constexpr (sm) {
    RT iDm[NS][NS], Xp[NS], nsum = RT(0);
#pragma unroll
    for (int s = 0; s < NS; ++s) nsum += Y[s] / RT(molar_mass(s));
#pragma unroll
    for (int s = 0, q = 0; s < NS; ++s)
#pragma unroll
      for (int r = s + 1; r < NS; ++r, ++q) {
        const RT v = Wp[(d.w_iD + q) * N + idx];
        iDm[s][r] = v;
        iDm[r][s] = v;
      }
#pragma unroll
    for (int s = 0; s < NS; ++s)
      Xp[s] = RT(CG ? Wd[(ND + 1 + s) * N + idx] : smem[(ND + 1 + s) * TILE_E + sidx]);
    RT A[NS][NS], Bm[NS][3], csum = RT(0);
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      RT diag = RT(0);
#pragma unroll
      for (int i = 0; i < NS; ++i) {
        if (i == s) continue;
        A[s][i] = Xp[s] * iDm[s][i];
        diag -= Xp[i] * iDm[s][i];
      }
      A[s][s] = diag;
      csum += fabs(diag);
    }
    const RT alpha = csum * RT(0.2);
#pragma unroll
    for (int i = 0; i < NS; ++i) {
      const RT am = alpha * (RT(molar_mass(i)) * nsum);
#pragma unroll
      for (int s = 0; s < NS; ++s) A[s][i] += am;
    }
    const RT bs = rho_r * nsum;
#pragma unroll
    for (int s = 0; s < NS; ++s)
#pragma unroll
      for (int b = 0; b < ND; ++b) Bm[s][b] = bs * dX[s][b];
    RT ip[NS];
#pragma unroll
    for (int k = 0; k < NS; ++k) {
      // pivot: the largest |A[i][k]|, i >= k, brought to row k by compare-and-swap
#pragma unroll
      for (int i = k + 1; i < NS; ++i) {
        const bool sw = fabs(A[i][k]) > fabs(A[k][k]);
#pragma unroll
        for (int c = k; c < NS; ++c) {
          const RT a = A[k][c], b = A[i][c];
          A[k][c] = sw ? b : a;
          A[i][c] = sw ? a : b;
        }
#pragma unroll
        for (int c = 0; c < ND; ++c) {
          const RT a = Bm[k][c], b = Bm[i][c];
          Bm[k][c] = sw ? b : a;
          Bm[i][c] = sw ? a : b;
        }
      }
      ip[k] = RT(1) / A[k][k];
#pragma unroll
      for (int i = k + 1; i < NS; ++i) {
        const RT l = A[i][k] * ip[k];
#pragma unroll
        for (int c = k + 1; c < NS; ++c) A[i][c] -= l * A[k][c];
#pragma unroll
        for (int c = 0; c < ND; ++c) Bm[i][c] -= l * Bm[k][c];
      }
    }
#pragma unroll
    for (int k = NS - 1; k >= 0; --k)
#pragma unroll
      for (int c = 0; c < ND; ++c) {
        RT v = Bm[k][c];
#pragma unroll
        for (int m = k + 1; m < NS; ++m) v -= A[k][m] * Bm[m][c];
        Bm[k][c] = v * ip[k];
      }
#pragma unroll
    for (int s = 0; s < NS; ++s)
#pragma unroll
      for (int c = 0; c < ND; ++c) Jsm[s][c] = RT(molar_mass(s)) * Bm[s][c];
  }
  // the 3-D flux planes (27 of them) are far larger than the last-level cache and are
  // stored nontemporal; the 2-D ones may still be cached when the divergence reads them
  auto put = [](double v, double* q) {
    if constexpr (ND == 3) st_once(v, q);
    else *q = v;
  };
#pragma unroll
  for (int j = 0; j < ND; ++j) {
    double* Fj = F + (long)j * nvar * N;
    RT J[NS];
    if (GAS == AIR5) {
      if (DX_PER_DIR) {
#pragma unroll
        for (int s = 0; s < NS; ++s) dX[s][j] = deriv(ND + 1 + s, j);
      }
      RT corr = RT(0);
      if constexpr (sm) {
#pragma unroll
        for (int s = 0; s < NS; ++s) J[s] = Jsm[s][j];
        if (AD) {
#pragma unroll
          for (int s = 0; s < NS; ++s) corr += a_s[s] * dX[s][j];
#pragma unroll
          for (int s = 0; s < NS; ++s) J[s] = J[s] - a_s[s] * dX[s][j] + Y[s] * corr;
        }
      } else {
#pragma unroll
        for (int s = 0; s < NS; ++s) corr += a_s[s] * dX[s][j];
#pragma unroll
        for (int s = 0; s < NS; ++s) J[s] = -a_s[s] * dX[s][j] + Y[s] * corr;
      }
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        // FP64: rho Y_s stands in for rho_s (equal to rounding; fewer live registers)
        const double rsj = sizeof(RT) == sizeof(double) ? rho * double(Y[s]) : rs[s];
        put(rsj * u[j] + double(J[s]), &Fj[s * N + idx]);
      }
    } else {
      put(rho * u[j], &Fj[idx]);
    }
    RT tau[3];
#pragma unroll
    for (int a = 0; a < ND; ++a) {
      RT t = mu_eff * (G[a][j] + G[j][a]);
      if (a == j) {
        t = t - mu_eff * RT(2.0 / 3.0) * theta;
        if (AD) t = t + beta * theta;
      }
      tau[a] = t;
      double conv = ld_once(&Q[(ns + a) * N + idx]) * u[j];
      if (a == j) conv = conv + pr;
      put(conv - double(t), &Fj[(ns + a) * N + idx]);
    }
    RT q = -kap_eff * dT[j];
    if (GAS == AIR5) {
      RT hJ = RT(0);
#pragma unroll
      for (int s = 0; s < NS; ++s) hJ += h[s] * J[s];
      q = q + hJ;
    }
    RT work = RT(0);
#pragma unroll
    for (int a = 0; a < ND; ++a) work += tau[a] * RT(u[a]);
    put((rhoE + pr) * u[j] - double(work - q), &Fj[(ns + ND) * N + idx]);
  }
}
template <int GAS, int ND, int ORDER, bool AD, class RT, bool SM = false>
__global__ __launch_bounds__(256) void k_flux(Dev d, const double* __restrict__ Q,
                                              const double* __restrict__ Wd,
                                              const RT* __restrict__ Wp,
                                              const RT* __restrict__ Gad, double* __restrict__ F) {
  flux_tile<GAS, ND, ORDER, AD, RT, SM, false, ND == 3 && AD && FLUX_ZFILTER>(d, Q, Wd, Wp, Gad,
                                                                            F);
}
// The same for FP64 on 2-D grids of at most two wavefronts per SIMD: occupancy is then
// bounded by the grid, not by registers, so the compiler may spend up to 256 VGPRs on
// instruction-level parallelism (measured: flat-plate flux -3 %; no gain in the mixed form).
template <int GAS, int ND, int ORDER, bool AD, class RT, bool SM = false>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 2))) void k_flux_small(
    Dev d, const double* __restrict__ Q, const double* __restrict__ Wd,
    const RT* __restrict__ Wp, const RT* __restrict__ Gad, double* __restrict__ F) {
  flux_tile<GAS, ND, ORDER, AD, RT, SM>(d, Q, Wd, Wp, Gad, F);
}

// The flux of the compact scheme: gradients from the line solves' planes.
template <int GAS, int ND, bool AD, class RT, bool SM = false>
__global__ __launch_bounds__(256) void k_flux_c(Dev d, const double* __restrict__ Q,
                                                const double* __restrict__ Wd,
                                                const RT* __restrict__ Wp,
                                                const RT* __restrict__ Gad,
                                                double* __restrict__ F,
                                                const double* __restrict__ Gc) {
  flux_tile<GAS, ND, 6, AD, RT, SM, true>(d, Q, Wd, Wp, Gad, F, Gc);
}

// ------------------------------------------------------------------ k_bc (wall row)
__constant__ double c_wall[4] = {48.0 / 25.0, -36.0 / 25.0, 16.0 / 25.0, -3.0 / 25.0};

// One wall point (i, k): no-slip velocity; temperature held (isothermal) or taken
// from the 4th-order extrapolation of the interior temperature (adiabatic, zero normal
// gradient); species mass fractions extrapolated likewise; the density already
// advanced by the stage is kept.  Held inflow points are left alone.
// get(v, m): component v of Q at row m = 1 .. 4 of the column (after the stage's update).
// TGET: get(nvar, m) returns the temperature of row m (thermally perfect gas: the rows'
// own threads inverted their energies side by side)
template <int GAS, int ND, class Get, bool TGET = false>
__device__ __forceinline__ void wall_point(const Dev& d, double* __restrict__ Q, int i, int k,
                                           Get get) {
  if (d.hold && d.hold[((long)k * 3 + 0) * d.nx + i]) return;
  const long N = d.N;
  const long idx0 = (long)k * d.ny * d.nx + i;
  constexpr int ns = (GAS == AIR5) ? NS : 1;
  if (GAS != AIR5) {
    const double rho_w = Q[idx0];
    const double ag = (d.gamma - 1.0) / d.gamma;
    double Tw;
    if (d.wall == HRX_WALL_ISOTHERMAL) {
      Tw = d.T_wall / d.T_ref;
    } else {
      Tw = 0.0;
#pragma unroll
      for (int m = 1; m <= 4; ++m) {
        const double rho = get(0, m);
        double ke = 0.0;
#pragma unroll
        for (int a = 0; a < ND; ++a) {
          const double ua = get(1 + a, m) / rho;
          ke += ua * ua;
        }
        const double e = get(1 + ND, m) / rho - 0.5 * ke;
        double Tm = d.gamma * e;
        if (GAS == TPG) {
          int status;
          Tm = TGET ? get(2 + ND, m)
                    : tpg_temperature(e, d.tpg_k0, d.tpg_th, ag, d.newton_rtol, d.newton_max,
                                      &status);
        }
        Tw += c_wall[m - 1] * Tm;
      }
    }
#pragma unroll
    for (int a = 0; a < ND; ++a) Q[(1 + a) * N + idx0] = 0.0;
    Q[(1 + ND) * N + idx0] =
        GAS == TPG ? rho_w * tpg_energy(Tw, d.tpg_k0, d.tpg_th, ag) : rho_w * Tw / d.gamma;
    return;
  }
  double rho_w = 0.0;
#pragma unroll
  for (int s = 0; s < NS; ++s) rho_w += Q[s * N + idx0];
  double Yw[NS] = {0.0, 0.0, 0.0, 0.0, 0.0};
  double Tw = 0.0;
  const double c2 = d.c_inf * d.c_inf;
#pragma unroll
  for (int m = 1; m <= 4; ++m) {
    double rho = 0.0, Y[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) rho += get(s, m);
    const double irho = 1.0 / rho;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      Y[s] = get(s, m) * irho;
      Yw[s] += c_wall[m - 1] * Y[s];
    }
    if (d.wall != HRX_WALL_ISOTHERMAL) {
      double ke = 0.0;
#pragma unroll
      for (int a = 0; a < ND; ++a) {
        const double ua = get(NS + a, m) * irho;
        ke += ua * ua;
      }
      const double e = get(NS + ND, m) * irho - 0.5 * ke;
      int status, iters;
      const double Tk = temperature_from_energy(e * c2, Y, d.newton_rtol, d.newton_max, &status,
                                                &iters);
      Tw += c_wall[m - 1] * (Tk / d.T_ref);
    }
  }
  if (d.wall == HRX_WALL_ISOTHERMAL) Tw = d.T_wall / d.T_ref;
#pragma unroll
  for (int s = 0; s < NS; ++s) Q[s * N + idx0] = rho_w * Yw[s];
#pragma unroll
  for (int a = 0; a < ND; ++a) Q[(ns + a) * N + idx0] = 0.0;
  const double ew = mixture_e(Tw * d.T_ref, Yw) / c2;
  Q[(ns + ND) * N + idx0] = rho_w * ew;
}

template <int GAS, int ND>
__global__ __launch_bounds__(128) void k_bc(Dev d, double* __restrict__ Q) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long nw = (long)(d.nx - 1) * d.nz;
  if (t >= nw) return;
  const int i = 1 + (int)(t % (d.nx - 1)), k = (int)(t / (d.nx - 1));
  const long idx0 = (long)k * d.ny * d.nx + i;
  wall_point<GAS, ND>(d, Q, i, k, [&](int v, int m) { return Q[v * d.N + idx0 + (long)m * d.nx]; });
}

// ------------------------------------------------------------------ k_div (+ RK)
// R = -sum_j dF_j/dx_j (FP64 differences, RT weighted sums) + wdot (species)
//     - sigma (Q - Q_ref) (FP64); boundary rows; then R out, or the low-storage update
// of Q and dQ in FP64.
// A block takes the chunks of KC components of its tile one after the other (PRE: each
// chunk's pointwise inputs loaded before its tiles are staged).  On small grids the
// chunks of a tile run side by side, so that more wavefronts are in flight: in 2-D in
// the two 256-thread halves of one block (NH = 2), in 3-D in one block per tile and
// chunk (chunk major: blocks [c nt, (c + 1) nt) take chunk c).  2-D tiles stage the x
// fluxes with their x halo and the y fluxes with their y halo; 3-D tiles lie in the
// (x, z) plane of one row (the order of the flux kernel) and stage the x and z fluxes,
// the y differences reading the neighbouring rows from memory.
// 2-D RK stages: the tiles of the bottom tile row (rows 0 .. TTY - 1) hold the four
// interior rows the wall condition extrapolates from, so their blocks apply it after the
// update (block barriers only) and no wall pass follows.
template <int GAS, int ND, int ORDER, int MODE, class RT, bool PRE, int NH>
__global__ __launch_bounds__(256 * NH) void k_div(Dev d, const double* __restrict__ F,
                                             const RT* __restrict__ Wp, const double* Qin,
                                             const double* __restrict__ Qref, double* Rout,
                                             double* Qio, double* dQio, double A, double B,
                                             double dt, int rkf) {
  constexpr int ns = (GAS == AIR5) ? NS : 1;
  constexpr int nvar = ns + ND + 1;
  constexpr int KC = div_chunk(ND);
  // 2-D RK stage: the wall condition runs here (see above), unless the tile's chunks run
  // in different blocks
  bool wall_in_div = ND == 2 && MODE == MODE_RK;
  // NH = 2: two halves of 256 threads update the two chunks of one tile side by side
  static_assert(NH == 1 || (ND == 2 && (nvar + KC - 1) / KC == 2), "two halves, two chunks");
  const int lt = NH == 1 ? (int)threadIdx.x : (int)(threadIdx.x & 255);
  const int half = NH == 1 ? 0 : (int)(threadIdx.x >> 8);
  extern __shared__ double smem_all[];
  double* smem = smem_all + half * KC * (FXE + FYE);
  const long N = d.N;
  Pt p;
  Sten sx, sy, sz;
  int i0 = 0, j0 = 0, k0t = 0, tx = 0, ty = 0;
  bool active = true;
  int kbeg = 0, kend = nvar;
  if (NH == 2) {
    kbeg = half * KC;
    kend = min(kbeg + KC, nvar);
  }
  {
    const unsigned nt = ND == 2 ? (unsigned)d.tgx * d.tgy : (unsigned)(d.tgx * d.tgz * d.ny);
    unsigned b = blockIdx.x, nb = gridDim.x;
    if (NH == 1 && gridDim.x > nt) {
      const unsigned c = blockIdx.x / nt;
      b -= c * nt;
      nb = nt;
      kbeg = (int)c * KC;
      kend = min(kbeg + KC, nvar);
      wall_in_div = false;
    }
    if (ND == 2) tile_origin(d, i0, j0, b, nb);
    else tile_origin3(d, i0, j0, k0t, b, nb);
    tx = lt & (TTX - 1);
    ty = lt / TTX;   // tile row: y in 2-D, z in 3-D
    p.i = i0 + tx;
    p.j = ND == 2 ? j0 + ty : j0;
    p.k = ND == 2 ? 0 : k0t + ty;
    // inactive threads still help stage the tiles
    active = p.i < d.nx && p.j < d.ny && p.k < d.nz;
    p.idx = ((long)p.k * d.ny + p.j) * d.nx + p.i;
    sx = make_sten<ORDER>((long)ty * TW + tx + THALO, 1, p.i, d.nx);
    if (ND == 2) {
      sy = make_sten<ORDER>((long)(ty + THALO) * TTX + tx, TTX, p.j, d.ny);
    } else {
      sy = make_sten<ORDER>(0, d.nx, p.j, d.ny);   // offsets from the point (row-uniform)
      sz = make_sten_central<ORDER>((long)(ty + THALO) * TTX + tx, TTX);
    }
  }
  const long idx = p.idx;
  const RT mx = active ? RT(d.mx[p.i]) : RT(0);
  const RT my = active ? RT(d.my[p.j]) : RT(0);
  const RT mz = (ND == 3 && active) ? RT(d.mz[p.k]) : RT(0);
  const double sig = active ? fmax(d.sx[p.i], d.sy[p.j]) : 0.0;
  bool held = (p.i == 0);
  if (active && d.hold && p.j < 3) held = held || d.hold[((long)p.k * 3 + p.j) * d.nx + p.i];
  constexpr int NPI = ORDER == 6 ? 3 : 2;
  // components in chunks of KC; each chunk's flux tiles are staged in LDS
  // PRE (2-D blocks that run several chunks): each chunk's pointwise inputs are loaded
  // before its tiles are staged, so that their latency overlaps the staging (each thread
  // reads only what it later writes); the production rates too in the mixed form.
  constexpr bool PRE_W = sizeof(RT) == sizeof(float);
  for (int k0 = kbeg; k0 < kend; k0 += KC) {
    const int kn = min(KC, kend - k0);
    double qv_[KC], dq_[KC];
    RT wd_[KC];
    if (PRE && active) {
#pragma unroll
      for (int kk = 0; kk < KC; ++kk) {
        const int k = min(k0 + kk, nvar - 1);
        qv_[kk] = (MODE == MODE_RK) ? Qio[k * N + idx] : Qin[k * N + idx];
        dq_[kk] = (MODE == MODE_RK && rkf != RKF_SSP_FIRST) ? dQio[k * N + idx] : 0.0;
        if (PRE_W) wd_[kk] = (GAS == AIR5 && k < NS) ? Wp[(d.w_wdot + k) * N + idx] : RT(0);
      }
    }
    {
      double* tx_ = smem;
      double* ty_ = smem + KC * FXE;
      if (k0 > kbeg) __syncthreads();   // previous chunk fully consumed
      // x-flux tiles of the chunk, then y-flux (2-D) or z-flux (3-D, periodic) tiles
      // (components past nvar read any valid plane and are never used)
      stage_tile<KC * FXE, TTX * TTY>(tx_, [&](int e) {
        const int kk = e / FXE, r = e - kk * FXE;
        const int ly = r / TW, lx = r - ly * TW;
        const int gi = min(max(i0 + lx - THALO, 0), d.nx - 1);
        const int k = min(k0 + kk, nvar - 1);
        if (ND == 2) {
          const int gj = min(j0 + ly, d.ny - 1);
          return F[(long)k * N + (long)gj * d.nx + gi];
        }
        const int gk = min(k0t + ly, d.nz - 1);
        return F[(long)k * N + ((long)gk * d.ny + j0) * d.nx + gi];
      }, lt);
      stage_tile<KC * FYE, TTX * TTY>(ty_, [&](int e) {
        const int kk = e / FYE, r = e - kk * FYE;
        const int ly = r / TTX, lx = r - ly * TTX;
        const int gi = min(i0 + lx, d.nx - 1);
        const int k = min(k0 + kk, nvar - 1);
        if (ND == 2) {
          const int gj = min(max(j0 + ly - THALO, 0), d.ny - 1);
          return F[((long)nvar + k) * N + (long)gj * d.nx + gi];
        }
        int gk = k0t + ly - THALO;
        gk = wrap_per(gk, d.nz);
        return F[((long)2 * nvar + k) * N + ((long)gk * d.ny + j0) * d.nx + gi];
      }, lt);
      __syncthreads();
    }
    if (!active) continue;
    // the component's update; qv_p, dq_p, wd_p are the preloaded inputs (PRE)
    auto update = [&](int kk, double qv_p, double dq_p, double wd_p) {
      const int k = k0 + kk;
      RT acc;
      if (ND == 2) {
        acc = sten_apply<RT>(sx, smem + kk * FXE) * mx;
        acc += sten_apply<RT>(sy, smem + KC * FXE + kk * FYE) * my;
      } else {
        acc = sten_apply<RT>(sx, smem + kk * FXE) * mx;
        acc += sten_apply<RT>(sy, F + ((long)nvar + k) * N + idx) * my;
        acc += sten_apply<RT, NPI>(sz, smem + KC * FXE + kk * FYE) * mz;
      }
      double R = -double(acc);
      if (GAS == AIR5 && k < NS)
        R = R + (PRE && PRE_W ? wd_p : double(Wp[(d.w_wdot + k) * N + idx]));
      const double qv = PRE ? qv_p : (MODE == MODE_RK) ? Qio[k * N + idx] : Qin[k * N + idx];
      if (Qref != nullptr && sig != 0.0) R = R - sig * (qv - Qref[k * N + idx]);
      if (held || (p.j == 0 && k >= ns && k < ns + ND)) R = 0.0;
      if (MODE == MODE_RHS) {
        Rout[k * N + idx] = R;
      } else {
        // the SSP form's first stage does not read the register (it is set to Q0)
        const double dqi =
            (PRE || rkf == RKF_SSP_FIRST) ? dq_p : dQio[k * N + idx];
        double qn, dqn;
        bool wdq;
        rk_update(rkf, A, B, dt, R, qv, dqi, qn, dqn, wdq);
        if (wdq) dQio[k * N + idx] = dqn;
        Qio[k * N + idx] = qn;
      }
    };
    if (PRE) {
#pragma unroll
      for (int kk = 0; kk < KC; ++kk)
        if (kk < kn) update(kk, qv_[kk], dq_[kk], PRE_W ? double(wd_[kk]) : 0.0);
    } else {
      for (int kk = 0; kk < kn; ++kk) update(kk, 0.0, 0.0, 0.0);
    }
  }
  if (wall_in_div && j0 == 0) {
    // rows 1 .. 4 of the updated state (each thread re-reads its own stores, each half
    // its own chunk) through LDS to the wall row's threads
    __syncthreads();   // the flux tiles in LDS are consumed
    if (active && ty >= 1 && ty <= 4) {
      for (int k = kbeg; k < kend; ++k) smem_all[(k * 4 + ty - 1) * TTX + tx] = Qio[k * N + idx];
      if (GAS == TPG && d.wall != HRX_WALL_ISOTHERMAL) {
        // the adiabatic wall extrapolates T: each row inverts its own energy
        const double rho = Qio[idx];
        double ke = 0.0;
#pragma unroll
        for (int a = 0; a < ND; ++a) {
          const double ua = Qio[(1 + a) * N + idx] / rho;
          ke += ua * ua;
        }
        const double e = Qio[(1 + ND) * N + idx] / rho - 0.5 * ke;
        int status;
        smem_all[(nvar * 4 + ty - 1) * TTX + tx] =
            tpg_temperature(e, d.tpg_k0, d.tpg_th, (d.gamma - 1.0) / d.gamma, d.newton_rtol,
                            d.newton_max, &status);
      }
    }
    __syncthreads();
    auto get = [&](int v, int m) { return smem_all[(v * 4 + m - 1) * TTX + tx]; };
    if (half == 0 && ty == 0 && p.i >= 1 && p.i < d.nx)
      wall_point<GAS, ND, decltype(get), GAS == TPG>(d, Qio, p.i, 0, get);
  }
}

// A first-derivative stencil over an LDS tile with 32-bit offsets (half the registers of
// Sten, which a march keeps live across its rows); same pairs, weights and order.
struct LSten {
  int p[4], q[4];
  double a[4];
};
__device__ __forceinline__ LSten lds_sten(const Sten& t) {
  LSten l;
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    l.p[m] = (int)t.p[m];
    l.q[m] = (int)t.q[m];
    l.a[m] = t.a[m];
  }
  return l;
}
template <class TA, int NP = 4>
__device__ __forceinline__ TA lsten_apply(const LSten& t, const double* f) {
  double d[NP];
#pragma unroll
  for (int m = 0; m < NP; ++m) d[m] = f[t.p[m]] - f[t.q[m]];
  TA acc = TA(t.a[0]) * TA(d[0]);
#pragma unroll
  for (int m = 1; m < NP; ++m) acc += TA(t.a[m]) * TA(d[m]);
  return acc;
}
// the central (periodic, staged) operator about LDS element b with stride s, as
// sten_apply<TA, NPI> over make_sten_central
template <int ORDER, class TA>
__device__ __forceinline__ TA lds_central(const double* f, int b, int s) {
  const double d0 = f[b + s] - f[b - s], d1 = f[b + 2 * s] - f[b - 2 * s];
  TA acc = TA(ORDER == 6 ? 0.75 : 2.0 / 3.0) * TA(d0);
  acc += TA(ORDER == 6 ? -0.15 : -1.0 / 12.0) * TA(d1);
  if (ORDER == 6) acc += TA(1.0 / 60.0) * TA(f[b + 3 * s] - f[b - 3 * s]);
  return acc;
}

// 3-D RK stage divergence as a march along y.  A block owns an (x, z) tile of TTX x TTY
// points, one chunk of KCM components and a segment of rows, and walks down the rows: the
// y fluxes of its points at rows j - H .. j + H (H = 3 for the sixth-order operator, 2
// for the fourth) ride in a register ring, one global read per value, where the
// row-per-block kernel reads every y neighbour from memory (six reads per value).  The x
// and z flux tiles of each row are staged in LDS as there, double-buffered: the next
// row's tile values are loaded into registers while the current row is computed (one
// block barrier per row).  Loads inside the march follow the rule of the AD march (the
// vector memory counter is waited on in order): the row's pointwise loads (the sponge's
// reference state only where the sponge acts) come first, then the ring's and the next
// tiles' loads, every one unconditional and consumed before its register is refilled.
// The differences are formed and weighted in the same order as the row-per-block kernel,
// so both give the same bits.  The four closure rows (0, 1, ny - 2, ny - 1) read their
// one-sided stencils from memory.
constexpr int KCM = 3;   // components per block of the march
template <int GAS, int ORDER, class RT>
__global__ __launch_bounds__(256) void k_div3m(Dev d, const double* __restrict__ F,
                                               const RT* __restrict__ Wp,
                                               const double* __restrict__ Qref, double* Qio,
                                               double* dQio, double A, double B, double dt,
                                               int rkf, int rseg, int nseg) {
  constexpr int ND = 3;
  constexpr int ns = (GAS == AIR5) ? NS : 1;
  constexpr int nvar = ns + ND + 1;
  constexpr int KC = KCM;
  constexpr int H = ORDER == 6 ? 3 : 2, NR = 2 * H + 1;
  constexpr int TOT = KC * (FXE + FYE);                  // one row's two flux tiles
  constexpr int NT = TTX * TTY, PER = (TOT + NT - 1) / NT;
  extern __shared__ double smem[];                       // two buffers of TOT
  const long N = d.N;
  const int nx = d.nx, ny = d.ny, nz = d.nz;
  // block -> (z tile fastest, x tile, row segment, chunk); each XCD takes a contiguous range
  const unsigned nb = gridDim.x, per = nb >> 3, b = blockIdx.x;
  unsigned t = b >= (per << 3) ? b : (b & 7u) * per + (b >> 3);
  const unsigned tgz = (unsigned)d.tgz, tgx = (unsigned)d.tgx;
  const int zt = (int)(t % tgz);
  t /= tgz;
  const int xt = (int)(t % tgx);
  t /= tgx;
  const int seg = (int)(t % (unsigned)nseg);
  const int chunk = (int)(t / (unsigned)nseg);
  const int i0 = xt * TTX, k0t = zt * TTY;
  const int kbeg = chunk * KC, kn = min(KC, nvar - kbeg);
  const int lt = threadIdx.x, tx = lt & (TTX - 1), ty = lt / TTX;
  const int pi = i0 + tx, pk = k0t + ty;
  const bool active = pi < nx && pk < nz;
  const int ci = min(pi, nx - 1), ck = min(pk, nz - 1);   // clamped (inactive threads)
  const int y0 = seg * rseg, y1 = min(y0 + rseg, ny);
  const long P = (long)nx * ny;
  const long col = (long)ck * P + ci;                       // point (ci, 0, ck)
  const RT mx = RT(d.mx[ci]), mz = RT(d.mz[ck]);
  const double sxi = d.sx[ci];
  const LSten sx = lds_sten(make_sten<ORDER>((long)ty * TW + tx + THALO, 1, ci, nx));
  const int zb = (ty + THALO) * TTX + tx;                   // the point in the z-flux tile
  // element e (clamped to the last one) of a row's tiles: x fluxes (x halo) then z
  // fluxes (periodic z halo); components past nvar read a valid plane, never used
  auto tile_src = [&](int e, int j) -> long {
    e = min(e, TOT - 1);
    if (e < KC * FXE) {
      const int kk = e / FXE, r = e - kk * FXE;
      const int ly = r / TW, lx = r - ly * TW;
      const int gi = min(max(i0 + lx - THALO, 0), nx - 1);
      const int gk = min(k0t + ly, nz - 1);
      return (long)min(kbeg + kk, nvar - 1) * N + ((long)gk * ny + j) * nx + gi;
    }
    e -= KC * FXE;
    const int kk = e / FYE, r = e - kk * FYE;
    const int ly = r / TTX, lx = r - ly * TTX;
    const int gi = min(i0 + lx, nx - 1);
    int gk = k0t + ly - THALO;
    gk = wrap_per(gk, nz);
    return ((long)2 * nvar + min(kbeg + kk, nvar - 1)) * N + ((long)gk * ny + j) * nx + gi;
  };
  double v[PER];
#pragma unroll
  for (int q = 0; q < PER; ++q) v[q] = F[tile_src(lt + q * NT, y0)];
  // the ring: y fluxes of rows j - H .. j + H (rows clamped to the grid); pf: the row
  // j + H + 1, loaded one row ahead
  double ry[KC][NR], pf[KC];
  auto fy = [&](int kk, int row) {
    const int k = min(kbeg + kk, nvar - 1);
    row = min(max(row, 0), ny - 1);
    return F[((long)nvar + k) * N + col + (long)row * nx];
  };
#pragma unroll
  for (int kk = 0; kk < KC; ++kk) {
#pragma unroll
    for (int m = 0; m < NR - 1; ++m) ry[kk][m] = fy(kk, y0 - H + m);
    pf[kk] = fy(kk, y0 + H);
  }
  const bool dq_in = rkf != RKF_SSP_FIRST;
  for (int j = y0; j < y1; ++j) {
    const long idx = col + (long)j * nx;
    double* buf = smem + (j & 1) * TOT;
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int e = lt + q * NT;
      if (e < TOT) buf[e] = v[q];
    }
    // the row's pointwise inputs (every one loaded; unused ones are discarded)
    const double sig = fmax(sxi, d.sy[j]);
    double qv_[KC], dq_[KC], qr_[KC];
    RT wd_[KC];
#pragma unroll
    for (int kk = 0; kk < KC; ++kk) {
      const int k = min(kbeg + kk, nvar - 1);
      qv_[kk] = ld_once(&Qio[k * N + idx]);
      dq_[kk] = ld_once(&dQio[k * N + idx]);
      wd_[kk] = GAS == AIR5 ? ld_once(&Wp[(d.w_wdot + min(k, NS - 1)) * N + idx]) : RT(0);
      qr_[kk] = 0.0;
      if (Qref != nullptr && sig != 0.0) qr_[kk] = Qref[k * N + idx];
    }
    // the ring's new row and the next row's tiles
#pragma unroll
    for (int kk = 0; kk < KC; ++kk) {
      ry[kk][NR - 1] = pf[kk];
      pf[kk] = fy(kk, j + H + 1);
    }
    // this row's buffer is complete, and every thread is done with the buffer the next
    // row overwrites (read two rows back)
    __syncthreads();
    const int jn = min(j + 1, ny - 1);
#pragma unroll
    for (int q = 0; q < PER; ++q) v[q] = F[tile_src(lt + q * NT, jn)];
    if (active) {
      const RT my = RT(d.my[j]);
      bool held = (pi == 0);
      if (d.hold && j < 3) held = held || d.hold[((long)pk * 3 + j) * nx + pi];
      // row class of the y operator: central sixth order (c6), central fourth order, or a
      // closure row read from memory
      const bool c6 = ORDER == 6 && j >= 3 && j <= ny - 4;
      const bool cen = c6 || (ORDER == 4 && j >= 2 && j <= ny - 3) ||
                       (ORDER == 6 && (j == 2 || j == ny - 3));
      const double a0 = c6 ? 0.75 : 2.0 / 3.0, a1 = c6 ? -0.15 : -1.0 / 12.0;
      const double a2 = c6 ? 1.0 / 60.0 : 0.0;
#pragma unroll
      for (int kk = 0; kk < KC; ++kk) {
        if (kk >= kn) continue;
        const int k = kbeg + kk;
        RT acc = lsten_apply<RT>(sx, buf + kk * FXE) * mx;
        RT ay;
        if (cen) {
          const double d0 = ry[kk][H + 1] - ry[kk][H - 1];
          const double d1 = ry[kk][H + 2] - ry[kk][H - 2];
          // the unused pairs difference the point with itself, as the stencil form does
          const double dc = ry[kk][H] - ry[kk][H];
          const double d2 = c6 ? ry[kk][NR - 1] - ry[kk][0] : dc;
          ay = RT(a0) * RT(d0);
          ay += RT(a1) * RT(d1);
          ay += RT(a2) * RT(d2);
          ay += RT(0.0) * RT(dc);
        } else {
          ay = sten_apply<RT>(make_sten<ORDER>(0, nx, j, ny), F + ((long)nvar + k) * N + idx);
        }
        acc += ay * my;
        acc += lds_central<ORDER, RT>(buf + KC * FXE + kk * FYE, zb, TTX) * mz;
        double R = -double(acc);
        if (GAS == AIR5 && k < NS) R = R + double(wd_[kk]);
        const double qv = qv_[kk];
        if (Qref != nullptr && sig != 0.0) R = R - sig * (qv - qr_[kk]);
        if (held || (j == 0 && k >= ns && k < ns + ND)) R = 0.0;
        double qn, dqn;
        bool wdq;
        rk_update(rkf, A, B, dt, R, qv, dq_in ? dq_[kk] : 0.0, qn, dqn, wdq);
        if (wdq) st_once(dqn, &dQio[k * N + idx]);
        st_once(qn, &Qio[k * N + idx]);
      }
    }
#pragma unroll
    for (int kk = 0; kk < KC; ++kk)
#pragma unroll
      for (int m = 0; m < NR - 1; ++m) ry[kk][m] = ry[kk][m + 1];
  }
}

// 3-D artificial-diffusivity sources |S| and theta (as k_ad_src) as a march along y, in
// the form of k_div3m: a block owns an (x, z) tile and a segment of rows; the velocity's
// y neighbours ride in a register ring, the (x, z) tiles with their halos are
// double-buffered in LDS, every load is unconditional and consumed before its register
// is refilled, and the derivatives are formed as in k_ad_src (same bits).
template <int ORDER, class RT>
__global__ __launch_bounds__(256) void k_ad_src3m(Dev d, const double* __restrict__ Wd,
                                                  RT* __restrict__ A, int rseg, int nseg) {
  constexpr int ND = 3;
  constexpr int H = ORDER == 6 ? 3 : 2, NR = 2 * H + 1;
  constexpr int TOT = ND * TILE_E;                       // u, v, w tiles of one row
  constexpr int NT = TTX * TTY, PER = (TOT + NT - 1) / NT;
  extern __shared__ double smem[];                       // two buffers of TOT
  const long N = d.N;
  const int nx = d.nx, ny = d.ny, nz = d.nz;
  // block -> (z tile fastest, x tile, row segment); each XCD takes a contiguous range
  const unsigned nb = gridDim.x, per = nb >> 3, b = blockIdx.x;
  unsigned t = b >= (per << 3) ? b : (b & 7u) * per + (b >> 3);
  const unsigned tgz = (unsigned)d.tgz, tgx = (unsigned)d.tgx;
  const int zt = (int)(t % tgz);
  t /= tgz;
  const int xt = (int)(t % tgx);
  const int seg = (int)(t / tgx);
  const int i0 = xt * TTX, k0t = zt * TTY;
  const int lt = threadIdx.x, tx = lt & (TTX - 1), ty = lt / TTX;
  const int pi = i0 + tx, pk = k0t + ty;
  const bool active = pi < nx && pk < nz;
  const int ci = min(pi, nx - 1), ck = min(pk, nz - 1);
  const int y0 = seg * rseg, y1 = min(y0 + rseg, ny);
  const long P = (long)nx * ny;
  const long col = (long)ck * P + ci;
  const RT mx = RT(d.mx[ci]), mz = RT(d.mz[ck]);
  const int sidx = (ty + THALO) * TW + tx + THALO;
  const LSten sx = lds_sten(make_sten<ORDER>(sidx, 1, ci, nx));
  auto tile_src = [&](int e, int j) -> long {
    e = min(e, TOT - 1);
    const int v = e / TILE_E, r = e - v * TILE_E;
    const int ly = r / TW, lx = r - ly * TW;
    const int gi = min(max(i0 + lx - THALO, 0), nx - 1);
    int gk = k0t + ly - THALO;
    gk = wrap_per(gk, nz);
    return (long)v * N + ((long)gk * ny + j) * nx + gi;
  };
  double vt[PER];
#pragma unroll
  for (int q = 0; q < PER; ++q) vt[q] = Wd[tile_src(lt + q * NT, y0)];
  double ry[ND][NR], pf[ND];
  auto fy = [&](int a, int row) {
    row = min(max(row, 0), ny - 1);
    return Wd[(long)a * N + col + (long)row * nx];
  };
#pragma unroll
  for (int a = 0; a < ND; ++a) {
#pragma unroll
    for (int m = 0; m < NR - 1; ++m) ry[a][m] = fy(a, y0 - H + m);
    pf[a] = fy(a, y0 + H);
  }
  for (int j = y0; j < y1; ++j) {
    const long idx = col + (long)j * nx;
    double* buf = smem + (j & 1) * TOT;
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int e = lt + q * NT;
      if (e < TOT) buf[e] = vt[q];
    }
#pragma unroll
    for (int a = 0; a < ND; ++a) {
      ry[a][NR - 1] = pf[a];
      pf[a] = fy(a, j + H + 1);
    }
    __syncthreads();
    const int jn = min(j + 1, ny - 1);
#pragma unroll
    for (int q = 0; q < PER; ++q) vt[q] = Wd[tile_src(lt + q * NT, jn)];
    if (active) {
      const RT my = RT(d.my[j]);
      const bool c6 = ORDER == 6 && j >= 3 && j <= ny - 4;
      const bool cen = c6 || (ORDER == 4 && j >= 2 && j <= ny - 3) ||
                       (ORDER == 6 && (j == 2 || j == ny - 3));
      const double a0 = c6 ? 0.75 : 2.0 / 3.0, a1 = c6 ? -0.15 : -1.0 / 12.0;
      const double a2 = c6 ? 1.0 / 60.0 : 0.0;
      RT G[3][3];
#pragma unroll
      for (int a = 0; a < ND; ++a) {
        const double* f = buf + a * TILE_E;
        G[a][0] = lsten_apply<RT>(sx, f) * mx;
        RT gy;
        if (cen) {
          const double d0 = ry[a][H + 1] - ry[a][H - 1];
          const double d1 = ry[a][H + 2] - ry[a][H - 2];
          const double dc = ry[a][H] - ry[a][H];
          const double d2 = c6 ? ry[a][NR - 1] - ry[a][0] : dc;
          gy = RT(a0) * RT(d0);
          gy += RT(a1) * RT(d1);
          gy += RT(a2) * RT(d2);
          gy += RT(0.0) * RT(dc);
        } else {
          gy = sten_apply<RT>(make_sten<ORDER>(0, nx, j, ny), Wd + (long)a * N + idx);
        }
        G[a][1] = gy * my;
        G[a][2] = lds_central<ORDER, RT>(f, sidx, TW) * mz;
      }
      RT s2 = RT(0);
#pragma unroll
      for (int a = 0; a < ND; ++a)
#pragma unroll
        for (int c = 0; c < ND; ++c) {
          const RT sab = RT(0.5) * (G[a][c] + G[c][a]);
          s2 += sab * sab;
        }
      RT theta = RT(0);
#pragma unroll
      for (int a = 0; a < ND; ++a) theta += G[a][a];
      A[0 * N + idx] = sqrt(s2);
      A[1 * N + idx] = theta;
    }
#pragma unroll
    for (int a = 0; a < ND; ++a)
#pragma unroll
      for (int m = 0; m < NR - 1; ++m) ry[a][m] = ry[a][m + 1];
  }
}

// Unfused stage update from a right-hand side R the caller computed: every component of
// every point, rk_update as in the divergence kernel (the wall row follows in k_bc).
__global__ __launch_bounds__(256) void k_rk_update(long N, int nvar, const double* __restrict__ R,
                                                   double* Q, double* dQ, double A, double B,
                                                   double dt, int rkf) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= N) return;
  for (int k = 0; k < nvar; ++k) {
    const long o = (long)k * N + idx;
    const double q = Q[o];
    const double dq = rkf == RKF_SSP_FIRST ? 0.0 : dQ[o];
    double qn, dqn;
    bool wdq;
    rk_update(rkf, A, B, dt, R[o], q, dq, qn, dqn, wdq);
    if (wdq) dQ[o] = dqn;
    Q[o] = qn;
  }
}

// ------------------------------------------------------------------ compact derivatives
// Collocated compact (Pade) first derivatives (Sec. 3.1 reading: the tridiagonal
// schemes of Lele's family).  Along a line of n points, A f' = r(f) with r formed from
// differences (unit spacing):
//   sixth-order interior rows (2 <= i <= n-3):  7/9 (f+1 - f-1) + 1/36 (f+2 - f-2)
//                                               A row (1/3, 1, 1/3)
//   Pade rows (the fourth-order interior; points 1, n-2 of the sixth-order scheme):
//                                               3/4 (f+1 - f-1),  A row (1/4, 1, 1/4)
//   end point 0:    2 (f1 - f0) + 1/2 (f2 - f0),             A row (1, 2)
//   end point n-1:  -(2 (f_{n-2} - f_{n-1}) + 1/2 (f_{n-3} - f_{n-1})), A row (2, 1)
//   periodic:       the interior row at every point, indices wrapped.
// The LU factors of A are the same for every line of a direction; the host forms them
// once: multipliers lo_i (L unit lower), U with super-diagonal up_i and reciprocal
// pivots iu_i.  Forward d_i = r_i - lo_i d_{i-1}; backward x_i = (d_i - up_i x_{i+1}) iu_i.
// The periodic direction solves the cyclic system by Sherman-Morrison: A = A' + u v^T,
// A' tridiagonal with corners (2, 1 + alpha^2), u = (-1, 0.., alpha), v = (1, 0.., -alpha);
// x = y - s (y_0 - alpha y_{n-1}) q with A' y = r, A' q = u, s = 1/(1 + v.q).
// (struct CLine: see above Dev)


// Right-hand side of row i from the values w[0..4] = f_{i-2} .. f_{i+2} (entries outside
// a non-periodic line are never read).
__device__ __forceinline__ double crow(const double* w, int i, int n, int order, bool per) {
  if (!per) {
    if (i == 0) return 2.0 * (w[3] - w[2]) + 0.5 * (w[4] - w[2]);
    if (i == n - 1) return -(2.0 * (w[1] - w[2]) + 0.5 * (w[0] - w[2]));
  }
  const bool six = order == 6 && (per || (i >= 2 && i <= n - 3));
  if (six) return (7.0 / 9.0) * (w[3] - w[1]) + (1.0 / 36.0) * (w[4] - w[0]);
  return 0.75 * (w[3] - w[1]);
}

// x lines: one wavefront per line, held in LDS (n <= CX_MAX).  Lane l owns the contiguous
// chunk [l C, (l + 1) C) of the line; each recurrence (forward, then backward) is a
// chain of affine maps, composed within the chunk, combined across the wavefront by a
// scan, then evaluated with the chunk's incoming value.  Planes p = blockIdx.y of f
// (stride fps) -> out (stride ops): out = scale m D f, or out += scale m D f (ACC).
constexpr int CX_MAX = 2048;
template <bool ACC>
__global__ __launch_bounds__(64) void k_cd_x(int n, const double* __restrict__ f, long fps,
                                             double* out, long ops, const double* __restrict__ m,
                                             double scale, int order, CLine L) {
  extern __shared__ double sm[];
  double* sf = sm;
  double* sd = sm + n;
  const int lane = threadIdx.x;
  const long line = blockIdx.x;
  const double* fl = f + (long)blockIdx.y * fps + line * n;
  double* ol = out + (long)blockIdx.y * ops + line * n;
  // loads in groups of eight per lane, all in flight before their LDS stores
  for (int i0 = 0; i0 < n; i0 += 512) {
    double v[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int i = i0 + lane + 64 * q;
      v[q] = i < n ? ld_once(&fl[i]) : 0.0;
    }
#pragma unroll
    for (int q = 0; q < 8; ++q)
      if (i0 + lane + 64 * q < n) sf[i0 + lane + 64 * q] = v[q];
  }
  __syncthreads();
  const int C = (n + 63) / 64;
  const int a = min(lane * C, n), b = min(a + C, n);
  auto rhs = [&](int i) {
    double w[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      const int q = i + k - 2;
      w[k] = (q >= 0 && q < n) ? sf[q] : 0.0;
    }
    return crow(w, i, n, order, false);
  };
  // forward: d_i = r_i - lo_i d_{i-1}; the chunk maps d_{a-1} to d_{b-1} as A x + B
  double A = 1.0, B = 0.0;
  for (int i = a; i < b; ++i) {
    const double li = L.lo[i];
    B = rhs(i) - li * B;
    A = -li * A;
  }
  for (int off = 1; off < 64; off <<= 1) {
    const double Ap = __shfl_up(A, off), Bp = __shfl_up(B, off);
    if (lane >= off) {
      B = A * Bp + B;
      A = A * Ap;
    }
  }
  double prev = __shfl_up(B, 1);
  if (lane == 0) prev = 0.0;
  for (int i = a; i < b; ++i) {
    const double di = rhs(i) - L.lo[i] * prev;
    sd[i] = di;
    prev = di;
  }
  // backward: x_i = (d_i - up_i x_{i+1}) iu_i; the chunk maps x_b to x_a as A x + B
  A = 1.0;
  B = 0.0;
  for (int i = b - 1; i >= a; --i) {
    const double iu = L.iu[i], u = L.up[i];
    B = (sd[i] - u * B) * iu;
    A = -(u * iu) * A;
  }
  for (int off = 1; off < 64; off <<= 1) {
    const double An = __shfl_down(A, off), Bn = __shfl_down(B, off);
    if (lane + off < 64) {
      B = A * Bn + B;
      A = A * An;
    }
  }
  double next = __shfl_down(B, 1);
  if (lane == 63) next = 0.0;
  for (int i = b - 1; i >= a; --i) {
    const double xi = (sd[i] - L.up[i] * next) * L.iu[i];
    sf[i] = xi;
    next = xi;
  }
  __syncthreads();
  for (int i0 = 0; i0 < n; i0 += 512) {
    double o[8], mv[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int i = min(i0 + lane + 64 * q, n - 1);
      mv[q] = m[i];
      o[q] = ACC ? ld_once(&ol[i]) : 0.0;
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int i = i0 + lane + 64 * q;
      if (i < n) {
        const double v = scale * mv[q] * sf[i];
        st_once(ACC ? o[q] + v : v, &ol[i]);
      }
    }
  }
}

// The same solve with the chunk length a power of two C (>= the lines' n / 64), four
// wavefronts per block sharing the LU factors, and K lines per wavefront taken in turn:
// a lane holds points lane + 64 q of the line in registers and forms their right-hand
// sides with the neighbours taken from the lanes that hold them; the right-hand sides
// are kept transposed -- element e at slot (e mod C) 64 + e / C -- with the factors, so
// that the lanes stepping through their chunks touch 64 consecutive slots.  The next
// line's loads are issued before the current line's solve, and the metric is loaded once
// per wavefront.  Where C = n / 64 exactly (every line of 64 C points) the chunks are
// those of k_cd_x.
template <bool ACC, int C, int K>
__global__ __launch_bounds__(256) void k_cd_xp(int n, long nlines, const double* __restrict__ f,
                                               long fps, double* out, long ops,
                                               const double* __restrict__ m, double scale,
                                               int order, CLine L) {
  constexpr int S = 64 * C;
  constexpr int LC = C == 1 ? 0 : C == 2 ? 1 : C == 4 ? 2 : C == 8 ? 3 : 4;
  static_assert((1 << LC) == C, "C a power of two up to 16");
  extern __shared__ double sm[];
  const int nw = blockDim.x >> 6;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  double* slo = sm;
  double* sup = sm + S;
  double* siu = sm + 2 * S;
  double* sr = sm + (3 + w) * S;       // r, then d, then x, transposed
  auto slot = [](int e) { return (e & (C - 1)) * 64 + (e >> LC); };
  for (int e = threadIdx.x; e < n; e += blockDim.x) {
    const int q = slot(e);
    slo[q] = L.lo[e];
    sup[q] = L.up[e];
    siu[q] = L.iu[e];
  }
  const long line0 = ((long)blockIdx.x * nw + w) * K;   // this wavefront's K lines
  const double* fp = f + (long)blockIdx.y * fps;
  double* op = out + (long)blockIdx.y * ops;
  // the metric (the same for every line) and the first line, point lane + 64 q in v[q]
  double v[C], mv[C];
#pragma unroll
  for (int q = 0; q < C; ++q) {
    const int i = min(lane + 64 * q, n - 1);
    mv[q] = m[i];
    v[q] = ld_once(&fp[min(line0, nlines - 1) * n + i]);
  }
  __syncthreads();   // the factors, staged by the whole block
  for (int kk = 0; kk < K; ++kk) {
    const long line = min(line0 + kk, nlines - 1);   // lines past the end redo the last
    const bool live = line0 + kk < nlines;
    {
      // right-hand sides: the neighbours i -+ 1, 2 from the lanes that hold them (from the
      // previous or next q where they wrap past lane 0 or 63)
      double m2p = 0.0, m1p = 0.0;
      double m2 = __shfl(v[0], (lane - 2) & 63), m1 = __shfl(v[0], (lane - 1) & 63);
      double p1 = __shfl(v[0], (lane + 1) & 63), p2 = __shfl(v[0], (lane + 2) & 63);
#pragma unroll
      for (int q = 0; q < C; ++q) {
        double p1n = 0.0, p2n = 0.0;
        if (q + 1 < C) {
          p1n = __shfl(v[q + 1], (lane + 1) & 63);
          p2n = __shfl(v[q + 1], (lane + 2) & 63);
        }
        const int i = lane + 64 * q;
        if (i < n) {
          double wv[5];
          wv[0] = lane >= 2 ? m2 : m2p;
          wv[1] = lane >= 1 ? m1 : m1p;
          wv[2] = v[q];
          wv[3] = lane <= 62 ? p1 : p1n;
          wv[4] = lane <= 61 ? p2 : p2n;
          sr[slot(i)] = crow(wv, i, n, order, false);
        }
        if (q + 1 < C) {
          m2p = m2;
          m1p = m1;
          m2 = __shfl(v[q + 1], (lane - 2) & 63);
          m1 = __shfl(v[q + 1], (lane - 1) & 63);
          p1 = p1n;
          p2 = p2n;
        }
      }
    }
    // the next line's loads, in flight during this line's solve
    if (kk + 1 < K) {
      const long ln = min(line0 + kk + 1, nlines - 1);
#pragma unroll
      for (int q = 0; q < C; ++q) v[q] = ld_once(&fp[ln * n + min(lane + 64 * q, n - 1)]);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const int nk = max(0, min(C, n - lane * C));
    // forward: d_i = r_i - lo_i d_{i-1}; the chunk maps d_{a-1} to d_{b-1} as A x + B
    double A = 1.0, B = 0.0;
#pragma unroll
    for (int k = 0; k < C; ++k) {
      if (k < nk) {
        const double li = slo[k * 64 + lane];
        B = sr[k * 64 + lane] - li * B;
        A = -li * A;
      }
    }
    for (int off = 1; off < 64; off <<= 1) {
      const double Ap = __shfl_up(A, off), Bp = __shfl_up(B, off);
      if (lane >= off) {
        B = A * Bp + B;
        A = A * Ap;
      }
    }
    double prev = __shfl_up(B, 1);
    if (lane == 0) prev = 0.0;
#pragma unroll
    for (int k = 0; k < C; ++k) {
      if (k < nk) {
        const double di = sr[k * 64 + lane] - slo[k * 64 + lane] * prev;
        sr[k * 64 + lane] = di;
        prev = di;
      }
    }
    // backward: x_i = (d_i - up_i x_{i+1}) iu_i; the chunk maps x_b to x_a as A x + B
    A = 1.0;
    B = 0.0;
#pragma unroll
    for (int k = C - 1; k >= 0; --k) {
      if (k < nk) {
        const double iu = siu[k * 64 + lane], u = sup[k * 64 + lane];
        B = (sr[k * 64 + lane] - u * B) * iu;
        A = -(u * iu) * A;
      }
    }
    for (int off = 1; off < 64; off <<= 1) {
      const double An = __shfl_down(A, off), Bn = __shfl_down(B, off);
      if (lane + off < 64) {
        B = A * Bn + B;
        A = A * An;
      }
    }
    double next = __shfl_down(B, 1);
    if (lane == 63) next = 0.0;
#pragma unroll
    for (int k = C - 1; k >= 0; --k) {
      if (k < nk) {
        const double xi = (sr[k * 64 + lane] - sup[k * 64 + lane] * next) * siu[k * 64 + lane];
        sr[k * 64 + lane] = xi;
        next = xi;
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (live) {
      double* ol = op + line * n;
      double o[C];
#pragma unroll
      for (int q = 0; q < C; ++q) o[q] = ACC ? ld_once(&ol[min(lane + 64 * q, n - 1)]) : 0.0;
#pragma unroll
      for (int q = 0; q < C; ++q) {
        const int i = lane + 64 * q;
        if (i < n) {
          const double x = scale * mv[q] * sr[slot(i)];
          st_once(ACC ? o[q] + x : x, &ol[i]);
        }
      }
    }
    // every lane has read this line's results before the next line's are written
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
}

// y or z lines: one thread per line marching along it (threads of a block hold
// consecutive x columns: every access is coalesced).  Line c = (cx, c2): first point
// c2 * s2 + cx, n points at stride s.  The forward values go to W (out itself, or a
// temporary plane when accumulating), the backward sweep turns them into x; the periodic
// direction ends with the Sherman-Morrison correction.
template <bool ACC, bool PER>
__global__ __launch_bounds__(128) void k_cd_col(int n, long s, int ncx, int nc2, long s2,
                                                const double* __restrict__ f, long fps,
                                                double* out, long ops, double* W, long wps,
                                                const double* __restrict__ m, double scale,
                                                int order, CLine L) {
  const long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= (long)ncx * nc2) return;
  const long c2 = c / ncx, cx = c - c2 * ncx;
  const long base = c2 * s2 + cx;
  const double* fl = f + (long)blockIdx.y * fps + base;
  double* ol = out + (long)blockIdx.y * ops + base;
  double* wl = (ACC ? W + (long)blockIdx.y * wps : out + (long)blockIdx.y * ops) + base;
  auto F = [&](int q) {
    if (PER) q = q < 0 ? q + n : (q >= n ? q - n : q);
    return fl[(long)q * s];
  };
  double w[5];
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    const int q = k - 2;
    w[k] = (PER || (q >= 0 && q < n)) ? F(q) : 0.0;
  }
  double prev = 0.0;
  for (int i = 0; i < n; ++i) {
    const double di = crow(w, i, n, order, PER) - L.lo[i] * prev;
    wl[(long)i * s] = di;
    prev = di;
#pragma unroll
    for (int k = 0; k < 4; ++k) w[k] = w[k + 1];
    const int q = i + 3;
    w[4] = (PER || q < n) ? F(q) : 0.0;
  }
  double next = 0.0, ylast = 0.0;
  for (int i = n - 1; i >= 0; --i) {
    const double xi = (wl[(long)i * s] - L.up[i] * next) * L.iu[i];
    if (i == n - 1) ylast = xi;
    next = xi;
    if (PER) {
      wl[(long)i * s] = xi;
    } else {
      const double v = scale * m[i] * xi;
      ol[(long)i * s] = ACC ? ol[(long)i * s] + v : v;
    }
  }
  if (PER) {
    const double fac = L.s * (next - L.alpha * ylast);   // next = y_0
    for (int i = 0; i < n; ++i) {
      const double xi = wl[(long)i * s] - fac * L.q[i];
      const double v = scale * m[i] * xi;
      ol[(long)i * s] = ACC ? ol[(long)i * s] + v : v;
    }
  }
}

// The same y or z line solves with the lines held on chip: a block of four wavefronts
// takes 16 consecutive lines (x columns c0 .. c0 + 15, first point c2 * s2 + c0, stride s)
// of n <= 16 CL points.  The block stages them in LDS with row-wise (coalesced) loads;
// wavefront w then owns lines 4w .. 4w + 3, lane (p, l) = (lane mod 16, lane / 16) the
// chunk [p CL, (p + 1) CL) of line 4w + l.  Each lane forms its chunk's right-hand sides
// into registers, and the two recurrences run as in k_cd_xp (affine maps composed within
// the chunk, scanned across the line's 16 lanes, then evaluated); the periodic direction
// adds the Sherman-Morrison correction in registers.  The results go back to LDS and
// leave row-wise: f is read once and out written (ACC: read and written) once, where
// the thread-per-line march also writes and re-reads the forward values.  Line element
// (i, line) sits at slot (i mod CL) 64 + i / CL + 16 (line mod 4) of wavefront line / 4's
// region, so that a step of the 64 lanes touches 64 consecutive slots; the factors are
// held the same way ((i mod CL) 16 + i / CL).  f and out are streamed with the nontemporal
// hint.  Up to CL = 16 the registers are capped at four wavefronts per SIMD (measured:
// the 512 x 256 x 128 jet's y and z solves -6 %; CL = 32 would spill).
template <bool ACC, bool PER, int CL>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(CL <= 16 ? 4 : 1))) void k_cd_colp(int n, long s, int ncx, long s2,
                                                 const double* __restrict__ f, long fps,
                                                 double* out, long ops,
                                                 const double* __restrict__ m, double scale,
                                                 int order, CLine L) {
  constexpr int RG = 64 * CL;            // one wavefront's region (4 lines)
  constexpr int NF = PER ? 4 : 3;        // factor arrays (lo, up, iu, q)
  extern __shared__ double sm[];
  double* sf = sm;                       // 4 regions
  double* sfac = sm + 4 * RG;            // NF arrays of 16 CL
  const int ngx = (ncx + 15) >> 4;
  const long c2 = blockIdx.x / (unsigned)ngx;
  const int c0 = (int)(blockIdx.x - c2 * ngx) * 16;
  const long base = c2 * s2 + c0;
  const double* fl = f + (long)blockIdx.y * fps + base;
  double* ol = out + (long)blockIdx.y * ops + base;
  const int t = threadIdx.x;
  auto slot = [](int i, int line) {
    return (line >> 2) * RG + (i & (CL - 1)) * 64 + (i / CL) + 16 * (line & 3);
  };
  // stage: element e = row * 16 + column (columns past ncx repeat the last one)
  constexpr int PER_T = CL;              // 16 CL rows x 16 columns / 256 threads
  double v[PER_T];
#pragma unroll
  for (int q = 0; q < PER_T; ++q) {
    const int e = t + 256 * q, row = min(e >> 4, n - 1), col = min(e & 15, ncx - 1 - c0);
    v[q] = ld_once(&fl[(long)row * s + col]);
  }
  for (int i = t; i < n; i += 256) {
    const int fs = (i & (CL - 1)) * 16 + i / CL;
    sfac[fs] = L.lo[i];
    sfac[16 * CL + fs] = L.up[i];
    sfac[32 * CL + fs] = L.iu[i];
    if (PER) sfac[48 * CL + fs] = L.q[i];
  }
#pragma unroll
  for (int q = 0; q < PER_T; ++q) {
    const int e = t + 256 * q;
    if ((e >> 4) < n) sf[slot(e >> 4, e & 15)] = v[q];
  }
  __syncthreads();
  const int w = t >> 6, lane = t & 63, p = lane & 15;
  const double* fw = sf + w * RG + (lane & 48);   // this lane's line, p added per row
  // value of row q of the lane's line (q in [-2, n + 1]; periodic rows wrap, rows outside
  // a non-periodic line are never used and read as 0)
  auto at = [&](int q) -> double {
    if (PER) q = q < 0 ? q + n : (q >= n ? q - n : q);
    else if (q < 0 || q >= n) return 0.0;
    return fw[(q & (CL - 1)) * 64 + q / CL];
  };
  const int a = p * CL, nk = max(0, min(CL, n - a));
  double r[CL];
  {
    // rows a - 2 .. a + nk + 1 only (an empty chunk reads nothing)
    double win[5];
#pragma unroll
    for (int k = 0; k < 4; ++k) win[k + 1] = nk > 0 ? at(a + k - 2) : 0.0;
#pragma unroll
    for (int k = 0; k < CL; ++k) {
#pragma unroll
      for (int j = 0; j < 4; ++j) win[j] = win[j + 1];
      win[4] = k < nk ? at(a + k + 2) : 0.0;
      r[k] = k < nk ? crow(win, a + k, n, order, PER) : 0.0;
    }
  }
  const double* flo = sfac + p;
  const double* fup = sfac + 16 * CL + p;
  const double* fiu = sfac + 32 * CL + p;
  // forward: d_i = r_i - lo_i d_{i-1}; the chunk maps d_{a-1} to d_{a+nk-1} as A x + B
  double A = 1.0, B = 0.0;
#pragma unroll
  for (int k = 0; k < CL; ++k) {
    if (k < nk) {
      const double li = flo[k * 16];
      B = r[k] - li * B;
      A = -li * A;
    }
  }
  for (int off = 1; off < 16; off <<= 1) {
    const double Ap = __shfl_up(A, off, 16), Bp = __shfl_up(B, off, 16);
    if (p >= off) {
      B = A * Bp + B;
      A = A * Ap;
    }
  }
  double prev = __shfl_up(B, 1, 16);
  if (p == 0) prev = 0.0;
#pragma unroll
  for (int k = 0; k < CL; ++k) {
    if (k < nk) {
      r[k] = r[k] - flo[k * 16] * prev;
      prev = r[k];
    }
  }
  // backward: x_i = (d_i - up_i x_{i+1}) iu_i; the chunk maps x_{a+nk} to x_a as A x + B
  A = 1.0;
  B = 0.0;
#pragma unroll
  for (int k = CL - 1; k >= 0; --k) {
    if (k < nk) {
      const double iu = fiu[k * 16], u = fup[k * 16];
      B = (r[k] - u * B) * iu;
      A = -(u * iu) * A;
    }
  }
  for (int off = 1; off < 16; off <<= 1) {
    const double An = __shfl_down(A, off, 16), Bn = __shfl_down(B, off, 16);
    if (p + off < 16) {
      B = A * Bn + B;
      A = A * An;
    }
  }
  double next = __shfl_down(B, 1, 16);
  if (p == 15) next = 0.0;
#pragma unroll
  for (int k = CL - 1; k >= 0; --k) {
    if (k < nk) {
      r[k] = (r[k] - fup[k * 16] * next) * fiu[k * 16];
      next = r[k];
    }
  }
  if (PER) {
    // x = y - s (y_0 - alpha y_{n-1}) q
    const int pl = (n - 1) / CL, kl = (n - 1) - pl * CL;
    double yl = 0.0;
#pragma unroll
    for (int k = 0; k < CL; ++k)
      if (k == kl) yl = r[k];
    const double y0 = __shfl(r[0], 0, 16);
    yl = __shfl(yl, pl, 16);
    const double fac = L.s * (y0 - L.alpha * yl);
    const double* fq = sfac + 48 * CL + p;
#pragma unroll
    for (int k = 0; k < CL; ++k)
      if (k < nk) r[k] = r[k] - fac * fq[k * 16];
  }
  // every lane of the wavefront has read its neighbours' rows: results overwrite them
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  {
    double* xw = sf + w * RG + lane;
#pragma unroll
    for (int k = 0; k < CL; ++k)
      if (k < nk) xw[k * 64] = r[k];
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < PER_T; ++q) {
    const int e = t + 256 * q, row = e >> 4, col = e & 15;
    if (row < n && c0 + col < ncx) {
      const double x = scale * m[row] * sf[slot(row, col)];
      double* o = ol + (long)row * s + col;
      st_once(ACC ? ld_once(o) + x : x, o);
    }
  }
}

// k_cd_colp: the chunk length, the power of two >= n / 16 (up to 32: 80 KB of LDS)
int cdcol_chunk(int n) {
  int c = 1;
  while (16 * c < n) c *= 2;
  return c;
}
bool cdcol_fits(int n) { return n >= 2 && n <= 512; }
// the thread-per-line solve (lines over 512 points) keeps its forward values in nvar
// temporary planes when it accumulates
bool cd_needs_temp(const Dev& d) {
  return d.compact && !(cdcol_fits(d.ny) && (d.ndim < 3 || cdcol_fits(d.nz)));
}

// Artificial-diffusivity sources |S| and theta of the compact scheme, pointwise from the
// velocity-gradient planes Gc[b][a].
template <int ND, class RT>
__global__ __launch_bounds__(256) void k_ad_src_c(Dev d, const double* __restrict__ Gc,
                                                  RT* __restrict__ A) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= d.N) return;
  const long N = d.N;
  RT G[3][3];
#pragma unroll
  for (int a = 0; a < ND; ++a)
#pragma unroll
    for (int b = 0; b < ND; ++b) G[a][b] = RT(Gc[((long)b * d.nsrc + a) * N + idx]);
  RT s2 = RT(0);
#pragma unroll
  for (int a = 0; a < ND; ++a)
#pragma unroll
    for (int b = 0; b < ND; ++b) {
      const RT sab = RT(0.5) * (G[a][b] + G[b][a]);
      s2 += sab * sab;
    }
  RT theta = RT(0);
#pragma unroll
  for (int a = 0; a < ND; ++a) theta += G[a][a];
  A[0 * N + idx] = sqrt(s2);
  A[1 * N + idx] = theta;
}

// The compact scheme's pointwise pass: R = Racc (the divergence, -sum_j D_j F_j) + wdot -
// sigma (Q - Q_ref), the held rows, then R out or the stage update (the wall row follows
// in k_bc).
template <int GAS, int ND, int MODE, class RT>
__global__ __launch_bounds__(256) void k_fin(Dev d, const RT* __restrict__ Wp, const double* Qin,
                                             const double* __restrict__ Qref, const double* Racc,
                                             double* Rout, double* Qio, double* dQio, double A,
                                             double B, double dt, int rkf) {
  constexpr int ns = (GAS == AIR5) ? NS : 1;
  constexpr int nvar = ns + ND + 1;
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= d.N) return;
  const long N = d.N;
  const Pt p = point_of(d, idx);
  const double sig = fmax(d.sx[p.i], d.sy[p.j]);
  bool held = p.i == 0;
  if (d.hold && p.j < 3) held = held || d.hold[((long)p.k * 3 + p.j) * d.nx + p.i];
#pragma unroll
  for (int k = 0; k < nvar; ++k) {
    double R = ld_once(&Racc[k * N + idx]);
    if (GAS == AIR5 && k < NS) R = R + double(ld_once(&Wp[(d.w_wdot + k) * N + idx]));
    const double qv = (MODE == MODE_RK) ? ld_once(&Qio[k * N + idx]) : ld_once(&Qin[k * N + idx]);
    if (Qref != nullptr && sig != 0.0) R = R - sig * (qv - Qref[k * N + idx]);
    if (held || (p.j == 0 && k >= ns && k < ns + ND)) R = 0.0;
    if (MODE == MODE_RHS) {
      Rout[k * N + idx] = R;
    } else {
      const double dq = rkf == RKF_SSP_FIRST ? 0.0 : ld_once(&dQio[k * N + idx]);
      double qn, dqn;
      bool wdq;
      rk_update(rkf, A, B, dt, R, qv, dq, qn, dqn, wdq);
      if (wdq) st_once(dqn, &dQio[k * N + idx]);
      st_once(qn, &Qio[k * N + idx]);
    }
  }
}

// ------------------------------------------------------------------ pointwise SI calls
// One SI state (rho, e, Y): energy inversion (from T_start in (T_MIN, T_GUESS_MAX), else
// cold), pressure, enthalpies, and transport from the surrogate's outputs ys = (ln T,
// ln mu, ln kappa, ln(rho D_s)) when net is set, else the plain evaluation.  Null
// outputs are skipped.  ld: leading dimension of the [5][.] arrays.  A non-finite input
// or rho <= 0 gives status 3 (counted) and NaN outputs.
template <class RT>
__device__ __forceinline__ void thermo_point(long ld, long i, double rtol, int max_iter,
                                             double r, double ee, const double* Y,
                                             double T_start, bool net,
                                             const float (&ys)[MLP_NOUT], double* Tout,
                                             double* pout, double* hout, double* muout,
                                             double* kout, double* Dout, int32_t* stout,
                                             unsigned long long* counters) {
  const long n = ld;
  {
    double v[NS + 1];
#pragma unroll
    for (int s = 0; s < NS; ++s) v[s] = Y[s];
    v[NS] = ee;
    if (!finite_state(v, NS + 1, r)) {
      atomicAdd(cslot(counters, 3), 1ull);
      const double nan = __builtin_nan("");
      Tout[i] = nan;
      if (stout) stout[i] = 3;
      if (pout) pout[i] = nan;
      if (muout) muout[i] = nan;
      if (kout) kout[i] = nan;
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        if (hout) hout[s * n + i] = nan;
        if (Dout) Dout[s * n + i] = nan;
      }
      return;
    }
  }
  int status, iters;
  SpeciesThermo st;   // species state at the last Newton iterate (within rtol of T)
  const double T = temperature_from_energy(ee, Y, rtol, max_iter, &status, &iters, T_start, &st);
  if (status == 1) atomicAdd(cslot(counters, 0), 1ull);
  if (status == 2) atomicAdd(cslot(counters, 1), 1ull);
  if (status) species_e_cv(T, st);
  Tout[i] = T;
  if (stout) stout[i] = status;
  const double p = r * mixture_R(Y) * T;
  if (pout) pout[i] = p;
  if (hout) {
#pragma unroll
    for (int s = 0; s < NS; ++s) hout[s * n + i] = st.e[s] + gas_const(s) * T;
  }
  if (net) {
    // the network's logarithms carry ~1e-4 relative error: FP32 exponentials suffice
    if (muout) muout[i] = (double)__expf(ys[1]);
    if (kout) kout[i] = (double)__expf(ys[2]);
    if (Dout) {
      const float ir = (float)(1.0 / r);
#pragma unroll
      for (int s = 0; s < NS; ++s) Dout[s * n + i] = (double)(__expf(ys[3 + s]) * ir);
    }
  } else if (muout || kout || Dout) {
    double X[NS], nsum = 0.0;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      X[s] = Y[s] * (1.0 / molar_mass(s));
      nsum += X[s];
    }
    const double inv = 1.0 / nsum;
#pragma unroll
    for (int s = 0; s < NS; ++s) X[s] = X[s] * inv;
    Transport<RT> tr;
    mixture_transport<RT>(T, p, X, st.cv, tr);
    if (muout) muout[i] = double(tr.mu);
    if (kout) kout[i] = double(tr.kappa);
    if (Dout) {
#pragma unroll
      for (int s = 0; s < NS; ++s) Dout[s * n + i] = double(tr.D[s]);
    }
  }
}

// Plain form, or (SUR) the surrogate form's second pass reading the network's outputs
// ys[8][n] (NaN in ys[0]: outside the hull, plain evaluation, counted when transport is
// requested).  n points of arrays with leading dimension ld (SoA [5][ld] for Y, h, D).
// Tout is read first: a temperature in (T_MIN, T_GUESS_MAX) starts the inversion.
template <class RT, bool SUR = false>
__global__ __launch_bounds__(128) void k_thermo_eval(long n, long ld, double rtol, int max_iter,
                                                     const double* __restrict__ rho,
                                                     const double* __restrict__ e,
                                                     const double* __restrict__ Yin,
                                                     double* __restrict__ Tout,
                                                     double* __restrict__ pout,
                                                     double* __restrict__ hout,
                                                     double* __restrict__ muout,
                                                     double* __restrict__ kout,
                                                     double* __restrict__ Dout,
                                                     int32_t* __restrict__ stout,
                                                     unsigned long long* counters,
                                                     const float* __restrict__ ysin) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double Y[NS];
#pragma unroll
  for (int s = 0; s < NS; ++s) Y[s] = Yin[s * ld + i];
  float ys[MLP_NOUT] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  bool net = false;
  if (SUR) {
#pragma unroll
    for (int o = 0; o < MLP_NOUT; ++o) ys[o] = ysin[o * n + i];
    net = !isnan(ys[0]);
    if (!net && (muout || kout || Dout)) atomicAdd(cslot(counters, 2), 1ull);
  }
  // the caller's temperature if it is a valid start, else the network's, else cold
  const double Tc = Tout[i];
  const bool tc_ok = Tc > T_MIN && Tc < T_GUESS_MAX;
  const double Ts = tc_ok ? Tc : (net ? (double)__expf(ys[0]) : 0.0);
  thermo_point<RT>(ld, i, rtol, max_iter, rho[i], e[i], Y, Ts, net, ys, Tout, pout, hout, muout,
                   kout, Dout, stout, counters);
}

template <class RT>
__global__ __launch_bounds__(128) void k_chem_source(long n, const double* __restrict__ rho_s,
                                                     const double* __restrict__ T,
                                                     double* __restrict__ wdot) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double rs[NS];
  RT w[NS];
#pragma unroll
  for (int s = 0; s < NS; ++s) rs[s] = rho_s[s * n + i];
  double em1[3];
  vib_em1(T[i], em1);
  production_rates<RT>(rs, T[i], em1, w, T_HI_MIXED);
#pragma unroll
  for (int s = 0; s < NS; ++s) wdot[s * n + i] = double(w[s]);
}

// LTE compositions of n points: rho [n], T [n], xiN [n] (or the context's free-stream
// value when null) -> Y [5][n], status [n] (may be null); counted like the inversion.
__global__ __launch_bounds__(128) void k_equilibrium(long n, double rtol, int max_iter,
                                                     const double* __restrict__ rho,
                                                     const double* __restrict__ T,
                                                     const double* __restrict__ xiN, double xi0,
                                                     double* __restrict__ Y,
                                                     int32_t* __restrict__ stout,
                                                     unsigned long long* counters) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double y[NS];
  int status;
  equilibrium_composition(rho[i], T[i], xiN ? xiN[i] : xi0, rtol, max_iter, y, &status);
#pragma unroll
  for (int s = 0; s < NS; ++s) Y[s * n + i] = y[s];
  if (stout) stout[i] = status;
  if (status == 1) atomicAdd(cslot(counters, 0), 1ull);
  if (status == 3) atomicAdd(cslot(counters, 3), 1ull);
}

// ------------------------------------------------------------------ surrogate network
// theta (FP32 flat) -> swizzled BF16 weights for the matrix cores, FP32 biases, and a
// BF16-rounded FP32 copy of the weights in flat order for the backward pass.
__global__ __launch_bounds__(256) void k_mlp_pack(const float* __restrict__ theta,
                                                  uint16_t* __restrict__ wsw,
                                                  float* __restrict__ bias,
                                                  float* __restrict__ wq) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < MLP_SW_SIZE;
       i += gridDim.x * blockDim.x) {
    int L = 3;
    while (L > 0 && i < MLP_SW_OFF[L]) --L;
    const int r = i - MLP_SW_OFF[L];
    const int q = r & 7, lane = (r >> 3) & 63, mt = r >> 9;
    const int m = mt / MLP_KS[L], t = mt % MLP_KS[L];
    const int o = 32 * m + (lane & 31);
    // hidden-layer inputs come in the accumulator order of the previous layer
    const int k = L == 0 ? 16 * t + 8 * (lane >> 5) + q : mlp_hidden_unit(t, lane >> 5, q);
    // first layer: columns k and 7 + k both carry W1[o][k] (hi/lo input pairs)
    const int kk = (L == 0 && k >= MLP_NIN && k < 2 * MLP_NIN) ? k - MLP_NIN : k;
    float v = 0.0f;
    if (o < MLP_NOUT_L[L] && kk < MLP_NIN_L[L]) v = theta[MLP_OFF_W[L] + o * MLP_NIN_L[L] + kk];
    wsw[i] = f2bf(v);
  }
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < MLP_NPARAM;
       i += gridDim.x * blockDim.x) {
    bool is_b = false;
    int bo = 0;
    for (int L = 0; L < 4; ++L)
      if (i >= MLP_OFF_B[L] && i < MLP_OFF_B[L] + MLP_NOUT_L[L]) {
        is_b = true;
        bo = (L == 0 ? 0 : (L == 1 ? 64 : (L == 2 ? 128 : 192))) + (i - MLP_OFF_B[L]);
      }
    wq[i] = is_b ? theta[i] : bf2f(f2bf(theta[i]));
    if (is_b) bias[bo] = theta[i];
  }
}

// Forward pass of n standardised inputs X [n][7] (rows gathered through idx when
// given) -> Y [n][8]; save != null keeps the hidden activations [3][n][64] (FP32).
__global__ __launch_bounds__(256) void k_mlp_fwd(long n, const float* __restrict__ X,
                                                 const int32_t* __restrict__ idx,
                                                 float* __restrict__ Y, float* save,
                                                 const uint16_t* __restrict__ gW,
                                                 const float* __restrict__ gB) {
  __shared__ __attribute__((aligned(16))) uint16_t sW[MLP_SW_SIZE];
  __shared__ float sB[MLP_NBIAS];
  __shared__ __attribute__((aligned(16))) uint16_t sH[4][64 * MLP_HPITCH];
  mlp_load_lds(gW, gB, sW, sB);
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (long base = (long)blockIdx.x * 256 + wave * 64; base < n; base += (long)gridDim.x * 256) {
    const long p = base + lane;
    const bool valid = p < n;
    float x[MLP_NIN], y[MLP_NOUT];
    const long row = valid ? (idx ? (long)idx[p] : p) : 0;
#pragma unroll
    for (int k = 0; k < MLP_NIN; ++k) x[k] = valid ? X[row * MLP_NIN + k] : 0.0f;
    mlp_wave64(sW, sB, sH[wave], x, y, save, base, n, valid);
    if (valid) {
#pragma unroll
      for (int o = 0; o < MLP_NOUT; ++o) Y[p * MLP_NOUT + o] = y[o];
    }
  }
}

// MSE over n x 8 outputs: dY = 2 (Y - T) / (8 n); loss += mean squared error.
__global__ __launch_bounds__(256) void k_mlp_mse(long n, const float* __restrict__ Y,
                                                 const float* __restrict__ T,
                                                 const int32_t* __restrict__ idx,
                                                 float* __restrict__ dY, float* loss) {
  __shared__ float red[256];
  const long m = n * MLP_NOUT;
  float acc = 0.0f;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < m;
       i += (long)gridDim.x * blockDim.x) {
    const long b = i / MLP_NOUT;
    const int o = (int)(i % MLP_NOUT);
    const long tb = idx ? (long)idx[b] : b;
    const float r = Y[i] - T[tb * MLP_NOUT + o];
    dY[i] = 2.0f * r / (float)m;
    acc += r * r;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0 && loss) atomicAdd(loss, red[0] / (float)m);
}

// Back-propagated deltas, one sample per thread: delta [n][200] = (d1, d2, d3, d4).
__global__ __launch_bounds__(128) void k_mlp_bwd_delta(long n, const float* __restrict__ dY,
                                                       const float* __restrict__ save,
                                                       const float* __restrict__ wq,
                                                       float* __restrict__ delta) {
  const long b = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= n) return;
  float* db = delta + b * 200;
  float d4[MLP_NOUT];
#pragma unroll
  for (int o = 0; o < MLP_NOUT; ++o) {
    d4[o] = dY[b * MLP_NOUT + o];
    db[192 + o] = d4[o];
  }
  float d3[64], d2[64];
  const float* W4 = wq + MLP_OFF_W[3];
#pragma unroll
  for (int k = 0; k < 64; ++k) {
    float sacc = 0.0f;
#pragma unroll
    for (int o = 0; o < MLP_NOUT; ++o) sacc += d4[o] * W4[o * 64 + k];
    const float a = save[(2 * n + b) * 64 + k];
    d3[k] = sacc * (2.0f * sqrtf(a));
    db[128 + k] = d3[k];
  }
  const float* W3 = wq + MLP_OFF_W[2];
#pragma unroll
  for (int k = 0; k < 64; ++k) {
    float sacc = 0.0f;
#pragma unroll
    for (int o = 0; o < 64; ++o) sacc += d3[o] * W3[o * 64 + k];
    const float a = save[(1 * n + b) * 64 + k];
    d2[k] = sacc * (2.0f * sqrtf(a));
    db[64 + k] = d2[k];
  }
  const float* W2 = wq + MLP_OFF_W[1];
#pragma unroll
  for (int k = 0; k < 64; ++k) {
    float sacc = 0.0f;
#pragma unroll
    for (int o = 0; o < 64; ++o) sacc += d2[o] * W2[o * 64 + k];
    const float a = save[(0 * n + b) * 64 + k];
    db[k] = sacc * (2.0f * sqrtf(a));
  }
}

// Weight and bias gradients, sum over the batch of delta_L[b][o] a_{L-1}[b][k] (a = the
// layer's BF16-rounded input as the forward pass used it; a_k = 1 for the bias).  Block
// (c, L) sums the batch chunk [c cb, (c + 1) cb) for layer L, staging 32 points at a
// time in LDS; thread t holds the products of output o = t mod O and inputs
// k = t / O + (256 / O) j.  Partial sums go to part[c][param], summed in chunk order by
// k_mlp_wgrad_sum (a fixed order: the result does not depend on scheduling).
constexpr int WG_MAXCH = 64, WG_SB = 32;
__global__ __launch_bounds__(256) void k_mlp_wgrad(long n, long cb, const float* __restrict__ X,
                                                   const int32_t* __restrict__ idx,
                                                   const float* __restrict__ save,
                                                   const float* __restrict__ delta,
                                                   float* __restrict__ part) {
  __shared__ float sD[WG_SB][64];
  __shared__ float sA[WG_SB][65];
  const int L = blockIdx.y;
  const int O = L == 3 ? MLP_NOUT : MLP_NH, K = L == 0 ? MLP_NIN : MLP_NH;
  const int doff = 64 * L;
  const int t = threadIdx.x;
  const int ks = 256 / O;
  const int o = t % O, kq = t / O;
  constexpr int NJ = 17;   // ceil(65 / 4)
  float acc[NJ];
#pragma unroll
  for (int j = 0; j < NJ; ++j) acc[j] = 0.0f;
  const long b0 = (long)blockIdx.x * cb, b1 = min(n, b0 + cb);
  for (long s0 = b0; s0 < b1; s0 += WG_SB) {
    const int sb = (int)min((long)WG_SB, b1 - s0);
    for (int e = t; e < WG_SB * O; e += 256) {
      const int r = e / O, c = e - r * O;
      sD[r][c] = r < sb ? delta[(s0 + r) * 200 + doff + c] : 0.0f;
    }
    for (int e = t; e < WG_SB * (K + 1); e += 256) {
      const int r = e / (K + 1), c = e - r * (K + 1);
      float a = 0.0f;
      if (r < sb) {
        const long bb = s0 + r;
        if (c == K) a = 1.0f;
        else if (L == 0) a = split_bf(X[(idx ? (long)idx[bb] : bb) * MLP_NIN + c]);
        else a = bf2f(f2bf(save[((long)(L - 1) * n + bb) * 64 + c]));
      }
      sA[r][c] = a;
    }
    __syncthreads();
    for (int r = 0; r < sb; ++r) {
      const float dl = sD[r][o];
#pragma unroll
      for (int j = 0; j < NJ; ++j) {
        const int k = kq + ks * j;
        if (k <= K) acc[j] += dl * sA[r][k];
      }
    }
    __syncthreads();
  }
  float* pc = part + (long)blockIdx.x * MLP_NPARAM;
  const int offw = L == 0 ? MLP_OFF_W[0] : (L == 1 ? MLP_OFF_W[1] : (L == 2 ? MLP_OFF_W[2] : MLP_OFF_W[3]));
  const int offb = L == 0 ? MLP_OFF_B[0] : (L == 1 ? MLP_OFF_B[1] : (L == 2 ? MLP_OFF_B[2] : MLP_OFF_B[3]));
#pragma unroll
  for (int j = 0; j < NJ; ++j) {
    const int k = kq + ks * j;
    if (k < K) pc[offw + o * K + k] = acc[j];
    else if (k == K) pc[offb + o] = acc[j];
  }
}

__global__ __launch_bounds__(256) void k_mlp_wgrad_sum(int nch, const float* __restrict__ part,
                                                       float* __restrict__ grad) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= MLP_NPARAM) return;
  float acc = 0.0f;
  for (int c = 0; c < nch; ++c) acc += part[(long)c * MLP_NPARAM + p];
  grad[p] = acc;
}

// Adam (beta1 = 0.9, beta2 = 0.999, eps = 1e-8) on the FP32 master parameters.
__global__ __launch_bounds__(256) void k_adam(float* __restrict__ theta, float* __restrict__ m,
                                              float* __restrict__ v,
                                              const float* __restrict__ g, float lr, float bc1,
                                              float bc2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= MLP_NPARAM) return;
  const float gi = g[i];
  const float mi = 0.9f * m[i] + 0.1f * gi;
  const float vi = 0.999f * v[i] + 0.001f * gi * gi;
  m[i] = mi;
  v[i] = vi;
  theta[i] = theta[i] - lr * (mi / bc1) / (sqrtf(vi / bc2) + 1e-8f);
}

// Mass fractions this far below zero still count as inside the hull: central
// differences leave undershoots of this size where a species vanishes (shocks, the
// wall extrapolation), and the network sees them as the zero it was trained on.
constexpr double Y_NEG_TOL = 1e-3;

// Inputs of the network from an SI state; returns false outside the training hull
// (log10 rho outside [min, max], a negative mass fraction, e outside
// [sum Y e_s(T_lo), sum Y e_s(T_hi)], or the element-N mass fraction outside its range).
// Raw features of an SI state: (log10 rho, ln T_c, Y_1..Y_5) with T_c the energy over
// the heat capacity of fully excited modes, (e - sum Y_s h0_s/M_s) / sum Y_s c_s.
__device__ __forceinline__ void surrogate_features(double rho, double e, const double* Y,
                                                   float* f) {
  double ef = 0.0, cf = 0.0;
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    ef += Y[s] * (hf0_molar(s) / molar_mass(s));
    cf += Y[s] * (gas_const(s) * (is_diatomic(s) ? 3.5 : 1.5));
  }
  const double ex = e - ef;
  f[0] = __log10f((float)rho);
  f[1] = ex > 0.0 && cf > 0.0 ? __logf((float)ex / (float)cf) : 0.0f;
#pragma unroll
  for (int s = 0; s < NS; ++s) f[2 + s] = (float)Y[s];
}

__device__ __forceinline__ bool surrogate_inputs(const MlpNorm& nm, double rho, double e,
                                                 const double* Y, float* x) {
  float f[MLP_NIN];
  surrogate_features(rho, e, Y, f);
  double elo = 0.0, ehi = 0.0;
  bool ok = f[0] >= nm.log10rho_min && f[0] <= nm.log10rho_max;
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    elo += Y[s] * nm.e_lo[s];
    ehi += Y[s] * nm.e_hi[s];
    ok = ok && Y[s] >= -Y_NEG_TOL;
  }
  const double xiN = Y[0] + Y[2] * (molar_mass(3) / molar_mass(2)) + Y[3];
  ok = ok && e >= elo && e <= ehi && xiN >= nm.xiN_min && xiN <= nm.xiN_max;
#pragma unroll
  for (int k = 0; k < MLP_NIN; ++k) x[k] = ok ? (f[k] - nm.in_mean[k]) * nm.in_istd[k] : 0.0f;
  return ok;
}

// Raw features of n SI states, f [n][7] (FP32), for building training sets.
__global__ __launch_bounds__(256) void k_mlp_features(long n, const double* __restrict__ rho,
                                                      const double* __restrict__ e,
                                                      const double* __restrict__ Yin,
                                                      float* __restrict__ f) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double Y[NS];
#pragma unroll
  for (int s = 0; s < NS; ++s) Y[s] = Yin[s * n + i];
  float v[MLP_NIN];
  surrogate_features(rho[i], e[i], Y, v);
#pragma unroll
  for (int k = 0; k < MLP_NIN; ++k) f[i * MLP_NIN + k] = v[k];
}

// ---- training sets of the surrogate, prepared on the device
// Raw features f (FP64 copy of the network's inputs, surrogate_features in FP64) and raw
// targets t = (ln T, ln mu, ln kappa, ln(rho D_1..5)) of the plain FP64 evaluation (cold
// energy inversion) of n SI states, rows f [n][7], t [n][8]; status as thermo_eval.
__global__ __launch_bounds__(128) void k_mlp_dataset(long n, double rtol, int max_iter,
                                                     const double* __restrict__ rho,
                                                     const double* __restrict__ e,
                                                     const double* __restrict__ Yin,
                                                     double* __restrict__ F,
                                                     double* __restrict__ Tt,
                                                     int32_t* __restrict__ stout,
                                                     unsigned long long* counters) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double Y[NS];
#pragma unroll
  for (int s = 0; s < NS; ++s) Y[s] = Yin[s * n + i];
  const double r = rho[i], ee = e[i];
  double ef = 0.0, cf = 0.0;
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    ef += Y[s] * (hf0_molar(s) / molar_mass(s));
    cf += Y[s] * (gas_const(s) * (is_diatomic(s) ? 3.5 : 1.5));
  }
  F[i * MLP_NIN + 0] = log10(r);
  F[i * MLP_NIN + 1] = log((ee - ef) / cf);
#pragma unroll
  for (int s = 0; s < NS; ++s) F[i * MLP_NIN + 2 + s] = Y[s];
  const float ys0[MLP_NOUT] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  double T, mu, kap, D[NS];
  int32_t st;
  // one state through the plain evaluation (leading dimension 1: scalar outputs)
  thermo_point<double>(1, 0, rtol, max_iter, r, ee, Y, 0.0, false, ys0, &T, nullptr, nullptr,
                       &mu, &kap, D, &st, counters);
  if (stout) stout[i] = st;
  Tt[i * MLP_NOUT + 0] = log(T);
  Tt[i * MLP_NOUT + 1] = log(mu);
  Tt[i * MLP_NOUT + 2] = log(kap);
#pragma unroll
  for (int s = 0; s < NS; ++s) Tt[i * MLP_NOUT + 3 + s] = log(D[s] * r);
}

// Moments of a training set for the surrogate's composition, per wavefront (lane 0
// writes the wavefront's sums to part[wave][K]; the host adds the wavefronts):
//   MODE 0: sum f_k                        (K = 7)
//   MODE 1: sum (f_k - m_k)^2              (K = 7)
//   MODE 2: sum a_i a_j (i <= j), sum a_i t_o with a = (1, (f - m)/s)   (K = 36 + 64)
//   MODE 3: sum r_o with r = t - L a       (K = 8)
//   MODE 4: sum (r_o - rm_o)^2             (K = 8)
// sv (device): m [7], 1/s [7], L [8][8] (row o: coefficients of a), rm [8].
template <int MODE>
__global__ __launch_bounds__(256) void k_fit_moments(long n, const double* __restrict__ F,
                                                     const double* __restrict__ Tt,
                                                     const double* __restrict__ sv,
                                                     double* __restrict__ part) {
  constexpr int K = MODE < 2 ? MLP_NIN : (MODE == 2 ? 36 + 64 : MLP_NOUT);
  double acc[K];
#pragma unroll
  for (int k = 0; k < K; ++k) acc[k] = 0.0;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long)gridDim.x * blockDim.x) {
    double f[MLP_NIN];
#pragma unroll
    for (int k = 0; k < MLP_NIN; ++k) f[k] = F[i * MLP_NIN + k];
    if (MODE == 0) {
#pragma unroll
      for (int k = 0; k < MLP_NIN; ++k) acc[k] += f[k];
      continue;
    }
    if (MODE == 1) {
#pragma unroll
      for (int k = 0; k < MLP_NIN; ++k) {
        const double d = f[k] - sv[k];
        acc[k] += d * d;
      }
      continue;
    }
    double a[8];
    a[0] = 1.0;
#pragma unroll
    for (int k = 0; k < MLP_NIN; ++k) a[1 + k] = (f[k] - sv[k]) * sv[MLP_NIN + k];
    if (MODE == 2) {
      int q = 0;
#pragma unroll
      for (int p = 0; p < 8; ++p)
#pragma unroll
        for (int r = p; r < 8; ++r) acc[q++] += a[p] * a[r];
#pragma unroll
      for (int o = 0; o < MLP_NOUT; ++o) {
        const double t = Tt[i * MLP_NOUT + o];
#pragma unroll
        for (int p = 0; p < 8; ++p) acc[36 + o * 8 + p] += a[p] * t;
      }
      continue;
    }
#pragma unroll
    for (int o = 0; o < MLP_NOUT; ++o) {
      double r = Tt[i * MLP_NOUT + o];
#pragma unroll
      for (int p = 0; p < 8; ++p) r -= sv[2 * MLP_NIN + o * 8 + p] * a[p];
      if (MODE == 3) {
        acc[o] += r;
      } else {
        const double d = r - sv[2 * MLP_NIN + 64 + o];
        acc[o] += d * d;
      }
    }
  }
  const long wave = ((long)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    double v = acc[k];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off);
    if ((threadIdx.x & 63) == 0) part[wave * K + k] = v;
  }
}

// Standardised training rows: x = (f - m)/s (FP32) and y = (t - L a - rm)/rs (FP32).
__global__ __launch_bounds__(256) void k_fit_apply(long n, const double* __restrict__ F,
                                                   const double* __restrict__ Tt,
                                                   const double* __restrict__ sv,
                                                   float* __restrict__ Xs,
                                                   float* __restrict__ Ys) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double a[8];
  a[0] = 1.0;
#pragma unroll
  for (int k = 0; k < MLP_NIN; ++k) {
    a[1 + k] = (F[i * MLP_NIN + k] - sv[k]) * sv[MLP_NIN + k];
    Xs[i * MLP_NIN + k] = (float)a[1 + k];
  }
#pragma unroll
  for (int o = 0; o < MLP_NOUT; ++o) {
    double r = Tt[i * MLP_NOUT + o];
#pragma unroll
    for (int p = 0; p < 8; ++p) r -= sv[2 * MLP_NIN + o * 8 + p] * a[p];
    Ys[i * MLP_NOUT + o] = (float)((r - sv[2 * MLP_NIN + 64 + o]) * sv[2 * MLP_NIN + 72 + o]);
  }
}

// network outputs -> (ln T, ln mu, ln kappa, ln(rho D_s)) (SI), FP32
__device__ __forceinline__ void surrogate_outputs(const MlpNorm& nm, const float* x,
                                                  const float* y, float* ys) {
#pragma unroll
  for (int o = 0; o < MLP_NOUT; ++o) {
    float v = nm.out_mean[o] + nm.out_std[o] * y[o] + nm.out_lin[o][0];
#pragma unroll
    for (int k = 0; k < MLP_NIN; ++k) v += nm.out_lin[o][1 + k] * x[k];
    ys[o] = v;
  }
}

// Network pass of the surrogate form.  A block of 4 wavefronts holds the network in
// LDS and walks the points in steps of 256; each wavefront computes the standardised
// features of its 64 states and evaluates the network on the matrix cores.  Output:
// ys[8][n] (FP32) = (ln T, ln mu, ln kappa, ln(rho D_1..5)) in SI, with ys[0] = NaN for
// states outside the training hull.  States are SI (rho, e, Y [5][ld]) or, with FROM_Q,
// the nondimensional conserved state Q.
template <int ND, bool FROM_Q>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void k_mlp_eval(Dev d, const MlpNorm* __restrict__ gnm, long n, long ld,
                                                  const double* __restrict__ rho,
                                                  const double* __restrict__ e,
                                                  const double* __restrict__ Yin,
                                                  const double* __restrict__ Q,
                                                  float* __restrict__ ysout,
                                                  const uint16_t* __restrict__ gW,
                                                  const float* __restrict__ gB) {
  __shared__ __attribute__((aligned(16))) uint16_t sW[MLP_SW_SIZE];
  __shared__ float sB[MLP_NBIAS];
  __shared__ __attribute__((aligned(16))) uint16_t sH[4][64 * MLP_HPITCH];
  // the composition statistics (about 0.5 KB) live in LDS next to the weights
  __shared__ __attribute__((aligned(16))) MlpNorm nm;
  mlp_load_lds(gW, gB, sW, sB);
  {
    const uint32_t* src = reinterpret_cast<const uint32_t*>(gnm);
    uint32_t* dst = reinterpret_cast<uint32_t*>(&nm);
    for (int k = threadIdx.x; k < (int)(sizeof(MlpNorm) / 4); k += blockDim.x) dst[k] = src[k];
  }
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (long base = (long)blockIdx.x * 256 + wave * 64; base < n; base += (long)gridDim.x * 256) {
    const long i = base + lane;
    const bool valid = i < n;
    const long ix = valid ? i : 0;
    double Y[NS], r, ee;
    if (FROM_Q) {
      double rs = 0.0;
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        Y[s] = Q[s * n + ix];
        rs += Y[s];
      }
      const double irs = 1.0 / rs;
#pragma unroll
      for (int s = 0; s < NS; ++s) Y[s] = Y[s] * irs;
      double ke = 0.0;
#pragma unroll
      for (int a = 0; a < ND; ++a) {
        const double ua = Q[(NS + a) * n + ix] * irs;
        ke += ua * ua;
      }
      r = rs * d.rho_inf;
      ee = (Q[(NS + ND) * n + ix] * irs - 0.5 * ke) * (d.c_inf * d.c_inf);
    } else {
#pragma unroll
      for (int s = 0; s < NS; ++s) Y[s] = Yin[s * ld + ix];
      r = rho[ix];
      ee = e[ix];
    }
    float x[MLP_NIN], y[MLP_NOUT], ys[MLP_NOUT];
    const bool in_hull = surrogate_inputs(nm, r, ee, Y, x) && valid;
    mlp_wave64(sW, sB, sH[wave], x, y, nullptr, 0, 0, valid);
    if (!valid) continue;
    surrogate_outputs(nm, x, y, ys);
    ysout[i] = in_hull ? ys[0] : __builtin_nanf("");
#pragma unroll
    for (int o = 1; o < MLP_NOUT; ++o) ysout[o * n + i] = ys[o];
  }
}

}  // namespace hrx

// ====================================================================== host side
using namespace hrx;

// Static device workspace of hrx_rhs_eval_noalloc: the scratch planes of one right-hand
// side (pointwise state, transport, artificial-diffusivity and flux planes) for callers
// that cannot allocate.  Every GPU the library runs on holds its own copy for the life
// of the process; calls on one GPU share it, so calls that overlap on one GPU race.
constexpr size_t NOALLOC_BYTES = (size_t)HRX_NOALLOC_MAX_BYTES;
static __device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

namespace {
constexpr int MAX_DEVICES = 64;
void* g_scratch[MAX_DEVICES] = {};
std::mutex g_scratch_mu;

// Device address of the current device's copy of scratch (the host-side name is only a
// stand-in): looked up once per device, with that device current.
int scratch_address(int dev, void** out) {
  if (dev < 0 || dev >= MAX_DEVICES) return HRX_EUNSUP;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return HRX_EHIP;
    g_scratch[dev] = p;
  }
  *out = g_scratch[dev];
  return HRX_OK;
}
}  // namespace

struct hrx_ctx {
  hrx_config cfg;
  Dev dev;
  hrx_reference ref;
  int nF;
  double *Wd = nullptr, *F = nullptr, *R = nullptr;
  double *G = nullptr, *Ct = nullptr;   // compact scheme: gradient planes, line temporaries
  double *cmat = nullptr;               // compact scheme: factors of the x, y, z lines
  void *Wp = nullptr, *AD = nullptr;   // RT planes (double, or float in the mixed form)
  int nWd = 0, nWp = 0;
  size_t rt_size = sizeof(double);
  double *metrics = nullptr;   // mx, my, mz, sx, sy, dlx, dly, dlz
  void* noalloc = nullptr;     // this device's copy of the static workspace (see scratch)
  unsigned char *hold = nullptr;
  unsigned long long *counters = nullptr;
  bool small_grid = false;   // at most two wavefronts per SIMD at one thread per point
  hipStream_t last_stream = nullptr;
  // kernel timing
  bool timing = false;
  std::vector<hipEvent_t> ev_free;
  struct Pending { int kid; hipEvent_t a, b; };
  std::vector<Pending> pending;
  double ms[HRX_NKERNELS] = {0};
  int64_t launches[HRX_NKERNELS] = {0};
  // surrogate network
  int thermo_mode = HRX_THERMO_PLAIN;
  bool mlp_params = false, mlp_norm = false;
  int64_t mlp_maxb = 0;
  float *theta = nullptr, *adam_m = nullptr, *adam_v = nullptr, *grad = nullptr;
  float *bias = nullptr, *wq = nullptr, *save = nullptr, *ybuf = nullptr, *dybuf = nullptr,
        *delta = nullptr, *wpart = nullptr;
  uint16_t* wsw = nullptr;
  double* fitbuf = nullptr;      // hrx_mlp_fit: statistics and per-wavefront moments
  MlpNorm* norm_dev = nullptr;   // composition statistics and hull (device copy)
  float* ys = nullptr;       // network outputs of the surrogate form, [8][ys_cap]
  int64_t ys_cap = 0;
  // replayable graphs of one RK stage, keyed by the call's arguments (non-null streams)
  struct StageGraph {
    const double *Q, *dQ, *Qref;
    double dt;
    int k;
    hipStream_t st;
    hipGraphExec_t exec;
  };
  std::vector<StageGraph> graphs;
  bool use_graphs = true;
};

namespace {

enum { K_PRIM = 0, K_AD_SRC, K_AD_D4, K_AD_FX, K_AD_FY, K_AD_FZ, K_FLUX, K_DIV, K_BC, K_THERMO,
       K_CHEM, K_CDERIV, K_FIN, K_EQUIL };


// Doubles of the surrogate fit's workspace: statistics, then 100 moments per wavefront of
// 256 blocks of 4 wavefronts (hrx_mlp_fit)
constexpr size_t FIT_DOUBLES = 2 * 7 + 64 + 2 * 8 + 256 * 4 * 100;

// Points per network pass of hrx_thermo_eval in the surrogate form (its workspace
// holds max(N, this) points; larger calls run in chunks).
constexpr int64_t THERMO_CHUNK = 1 << 20;

// Workspace of the surrogate's network outputs, [8][n] floats.  Sized once, by
// hrx_set_thermo_mode (a set-up call, which also drops every captured graph); the
// compute calls never grow it.
int ensure_ys(hrx_ctx* c, int64_t n) {
  if (n <= c->ys_cap) return HRX_OK;
  if (c->ys) (void)hipFree(c->ys);
  c->ys = nullptr;
  c->ys_cap = 0;
  if (hipMalloc(&c->ys, sizeof(float) * MLP_NOUT * (size_t)n) != hipSuccess) return HRX_ENOMEM;
  c->ys_cap = n;
  return HRX_OK;
}

int flush_timing(hrx_ctx* c) {
  for (auto& p : c->pending) {
    if (hipEventSynchronize(p.b) != hipSuccess) return HRX_EHIP;
    float t = 0.0f;
    if (hipEventElapsedTime(&t, p.a, p.b) != hipSuccess) return HRX_EHIP;
    c->ms[p.kid] += t;
    c->launches[p.kid] += 1;
    c->ev_free.push_back(p.a);
    c->ev_free.push_back(p.b);
  }
  c->pending.clear();
  return HRX_OK;
}

// Launch f() on stream st, bracketed by events when timing is on.
template <class Fn>
void timed(hrx_ctx* c, int kid, hipStream_t st, Fn&& f) {
  if (!c->timing) {
    f();
    return;
  }
  if (c->ev_free.size() < 2) flush_timing(c);
  if (c->ev_free.size() < 2) {
    f();
    return;
  }
  hipEvent_t a = c->ev_free.back(); c->ev_free.pop_back();
  hipEvent_t b = c->ev_free.back(); c->ev_free.pop_back();
  (void)hipEventRecord(a, st);
  f();
  (void)hipEventRecord(b, st);
  c->pending.push_back({kid, a, b});
}

}  // namespace

namespace {

// index-space first derivative of a host array (same operator as the kernels)
void host_deriv(const std::vector<double>& f, int order, std::vector<double>& out) {
  const int n = (int)f.size();
  out.assign(n, 0.0);
  const int h = order == 6 ? 3 : 2;
  for (int i = h; i < n - h; ++i) {
    double acc;
    if (order == 6) {
      acc = 0.75 * (f[i + 1] - f[i - 1]);
      acc += -0.15 * (f[i + 2] - f[i - 2]);
      acc += (1.0 / 60.0) * (f[i + 3] - f[i - 3]);
    } else {
      acc = (2.0 / 3.0) * (f[i + 1] - f[i - 1]);
      acc += (-1.0 / 12.0) * (f[i + 2] - f[i - 2]);
    }
    out[i] = acc;
  }
  const double b0[5] = {-25.0 / 12.0, 4.0, -3.0, 4.0 / 3.0, -0.25};
  const double b1[5] = {-0.25, -5.0 / 6.0, 1.5, -0.5, 1.0 / 12.0};
  double s0 = 0, s1 = 0, e0 = 0, e1 = 0;
  for (int m = 0; m < 5; ++m) {
    s0 += b0[m] * f[m];
    s1 += b1[m] * f[m];
    e0 += b0[m] * f[n - 1 - m];
    e1 += b1[m] * f[n - 1 - m];
  }
  out[0] = s0;
  out[1] = s1;
  out[n - 1] = -e0;
  out[n - 2] = -e1;
  if (order == 6) {
    for (int i : {2, n - 3}) {
      double acc = (2.0 / 3.0) * (f[i + 1] - f[i - 1]);
      acc += (-1.0 / 12.0) * (f[i + 2] - f[i - 2]);
      out[i] = acc;
    }
  }
}

// Host copy of the compact factors of one direction (the device copy goes to cmat).
struct HostCLine {
  std::vector<double> lo, up, iu, q;
  double s = 0.0, alpha = 0.0;
};

// LU factors of the compact matrix of a line of n points: the non-periodic matrix
// (end rows (1, 2) and (2, 1), Pade rows (1/4, 1, 1/4), sixth-order rows (1/3, 1, 1/3)),
// or for a periodic line the tridiagonal part A' of the cyclic matrix, with
// q = A'^-1 u, s = 1/(1 + v.q) (Sherman-Morrison, u = (-1, 0.., alpha),
// v = (1, 0.., -alpha)).
HostCLine compact_factors(int n, int order, bool per) {
  std::vector<double> sub(n, 0.0), dia(n, 1.0), sup(n, 0.0);
  HostCLine L;
  const double a6 = 1.0 / 3.0, a4 = 0.25;
  if (!per) {
    for (int i = 0; i < n; ++i) {
      if (i == 0) sup[i] = 2.0;
      else if (i == n - 1) sub[i] = 2.0;
      else if (order == 6 && i >= 2 && i <= n - 3) sub[i] = sup[i] = a6;
      else sub[i] = sup[i] = a4;
    }
  } else {
    const double al = order == 6 ? a6 : a4;
    for (int i = 0; i < n; ++i) sub[i] = sup[i] = al;
    sub[0] = 0.0;
    sup[n - 1] = 0.0;
    dia[0] = 2.0;
    dia[n - 1] = 1.0 + al * al;
    L.alpha = al;
  }
  L.lo.assign(n, 0.0);
  L.up = sup;
  L.iu.assign(n, 0.0);
  double u = dia[0];
  L.iu[0] = 1.0 / u;
  for (int i = 1; i < n; ++i) {
    L.lo[i] = sub[i] / u;
    u = dia[i] - L.lo[i] * L.up[i - 1];
    L.iu[i] = 1.0 / u;
  }
  if (per) {
    std::vector<double> r(n, 0.0);
    r[0] = -1.0;
    r[n - 1] = L.alpha;
    L.q.assign(n, 0.0);
    double prev = 0.0;
    for (int i = 0; i < n; ++i) { r[i] -= L.lo[i] * prev; prev = r[i]; }
    double next = 0.0;
    for (int i = n - 1; i >= 0; --i) { L.q[i] = (r[i] - L.up[i] * next) * L.iu[i]; next = L.q[i]; }
    L.s = 1.0 / (1.0 + L.q[0] - L.alpha * L.q[n - 1]);
  }
  return L;
}

// Compact first derivative (index space) of a host array on a non-periodic line.
void host_compact_deriv(const std::vector<double>& f, int order, const HostCLine& L,
                        std::vector<double>& out) {
  const int n = (int)f.size();
  out.assign(n, 0.0);
  double prev = 0.0;
  for (int i = 0; i < n; ++i) {
    double r;
    if (i == 0) r = 2.0 * (f[1] - f[0]) + 0.5 * (f[2] - f[0]);
    else if (i == n - 1) r = -(2.0 * (f[n - 2] - f[n - 1]) + 0.5 * (f[n - 3] - f[n - 1]));
    else if (order == 6 && i >= 2 && i <= n - 3)
      r = (7.0 / 9.0) * (f[i + 1] - f[i - 1]) + (1.0 / 36.0) * (f[i + 2] - f[i - 2]);
    else r = 0.75 * (f[i + 1] - f[i - 1]);
    out[i] = r - L.lo[i] * prev;
    prev = out[i];
  }
  double next = 0.0;
  for (int i = n - 1; i >= 0; --i) { out[i] = (out[i] - L.up[i] * next) * L.iu[i]; next = out[i]; }
}

int check(hipError_t e) { return e == hipSuccess ? HRX_OK : HRX_EHIP; }

inline unsigned blocks_for(long n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

extern "C" {

const char* hrx_strerror(int code) {
  switch (code) {
    case HRX_OK: return "ok";
    case HRX_EINVAL: return "invalid argument or configuration";
    case HRX_EHIP: return "HIP runtime error";
    case HRX_ENOMEM: return "device memory allocation failed";
    case HRX_EUNSUP: return "not supported by this library";
    case HRX_ENEWTON: return "the energy inversion did not converge at some point";
    case HRX_EDOMAIN: return "an energy below e(50 K) at some point";
    case HRX_ENONFINITE: return "a non-finite state or a non-positive density at some point";
    case HRX_ETOOBIG:
      return "the problem's scratch exceeds the static workspace of hrx_rhs_eval_noalloc";
    default: return "unknown error";
  }
}

static void clear_graphs(hrx_ctx* c) {
  for (auto& g : c->graphs) (void)hipGraphExecDestroy(g.exec);
  c->graphs.clear();
}

void hrx_destroy(hrx_ctx* c) {
  if (!c) return;
  clear_graphs(c);
  if (c->timing) hrx_timing_enable(c, 0);
  (void)hipFree(c->Wd);
  (void)hipFree(c->Wp);
  (void)hipFree(c->F);
  (void)hipFree(c->R);
  (void)hipFree(c->AD);
  (void)hipFree(c->metrics);
  (void)hipFree(c->G);
  (void)hipFree(c->Ct);
  (void)hipFree(c->cmat);
  (void)hipFree(c->hold);
  (void)hipFree(c->counters);
  (void)hipFree(c->ys);
  (void)hipFree(c->norm_dev);
  for (void* q : {(void*)c->theta, (void*)c->adam_m, (void*)c->adam_v, (void*)c->grad,
                  (void*)c->bias, (void*)c->wq, (void*)c->save, (void*)c->ybuf, (void*)c->dybuf,
                  (void*)c->delta, (void*)c->wpart, (void*)c->wsw, (void*)c->fitbuf})
    (void)hipFree(q);
  delete c;
}

int hrx_create(const hrx_config* cfg, hrx_ctx** out) {
  if (!cfg || !out) return HRX_EINVAL;
  *out = nullptr;
  const hrx_config& c = *cfg;
  if (c.gas != HRX_GAS_CPG && c.gas != HRX_GAS_AIR5 && c.gas != HRX_GAS_TPG) return HRX_EINVAL;
  if (c.diffusion != HRX_DIFF_RAMSHAW && c.diffusion != HRX_DIFF_STEFAN_MAXWELL) return HRX_EINVAL;
  if (c.diffusion == HRX_DIFF_STEFAN_MAXWELL && c.gas != HRX_GAS_AIR5) return HRX_EUNSUP;
  if (c.nx < 8 || c.ny < 8 || c.nz < 1 || (c.nz > 1 && c.nz < 8)) return HRX_EINVAL;
  if (c.fd_order != 4 && c.fd_order != 6) return HRX_EINVAL;
  if (c.fd_scheme != HRX_FD_EXPLICIT && c.fd_scheme != HRX_FD_COMPACT) return HRX_EINVAL;
  if (c.fd_scheme == HRX_FD_COMPACT && c.nx > CX_MAX) return HRX_EUNSUP;
  if (c.rk_scheme != HRX_RK3_2N && c.rk_scheme != HRX_RK45_2N && c.rk_scheme != HRX_SSPRK3)
    return HRX_EINVAL;
  if (c.precision != HRX_PREC_FP64 && c.precision != HRX_PREC_MIXED) return HRX_EINVAL;
  if (!c.x || !c.y || (c.nz > 1 && !c.z)) return HRX_EINVAL;
  if (c.sponge_in < 0 || c.sponge_out < 0 || c.sponge_top < 0 || c.sponge_in >= c.nx - 1 ||
      c.sponge_out >= c.nx - 1 || c.sponge_top >= c.ny - 1)
    return HRX_EINVAL;
  if (c.wall == HRX_WALL_ISOTHERMAL && !(c.T_wall > 0.0)) return HRX_EINVAL;
  if (!(c.T_inf > 0.0)) return HRX_EINVAL;
  const long N = (long)c.nx * c.ny * c.nz;
  for (int64_t h = 0; h < c.n_hold; ++h) {
    if (!c.hold || c.hold[h] < 0 || c.hold[h] >= N) return HRX_EINVAL;
    const long r = c.hold[h] / c.nx;
    if (r % c.ny >= 3) return HRX_EINVAL;
  }
  hrx_ctx* ctx = new (std::nothrow) hrx_ctx();
  if (!ctx) return HRX_ENOMEM;
  ctx->cfg = c;
  ctx->cfg.hold = nullptr;
  Dev& d = ctx->dev;
  std::memset(&d, 0, sizeof(d));
  const int nd = c.nz > 1 ? 3 : 2;
  const int ns = c.gas == HRX_GAS_AIR5 ? NS : 1;
  d.nx = c.nx; d.ny = c.ny; d.nz = c.nz; d.ndim = nd; d.ns = ns; d.nvar = ns + nd + 1;
  d.fd_order = c.fd_order; d.N = N;
  d.gx = (c.nx + TX - 1) / TX;
  d.tgx = (c.nx + TTX - 1) / TTX;
  d.tgy = (c.ny + TTY - 1) / TTY;
  d.tgz = (c.nz + TTY - 1) / TTY;
  d.newton_rtol = c.newton_rtol > 0.0 ? c.newton_rtol : 1e-13;
  d.newton_max = c.newton_max_iter > 0 ? c.newton_max_iter : 50;
  d.wall = c.wall; d.T_wall = c.T_wall;
  d.ad_on = c.ad_on ? 1 : 0;
  d.Cmu = c.ad_coef[0]; d.Cbeta = c.ad_coef[1]; d.Ckap = c.ad_coef[2]; d.CD = c.ad_coef[3];
  d.CY = c.ad_coef[4];
  // ---------------------------------------------------------- reference state (Eq. 7, 11)
  hrx_reference& ref = ctx->ref;
  std::memset(&ref, 0, sizeof(ref));
  if (c.gas == HRX_GAS_CPG) {
    if (!(c.gamma > 1.0) || !(c.Pr > 0.0) || !(c.Re > 0.0)) { delete ctx; return HRX_EINVAL; }
    ref.gamma = c.gamma; ref.Re = c.Re; ref.Pr = c.Pr; ref.Ec = 1.0;
    ref.T_ref = (c.gamma - 1.0) * c.T_inf;
    ref.mu_inf = sutherland<double>(c.T_inf);
  } else if (c.gas == HRX_GAS_TPG) {
    // Sec. 2.2.2: c_p0 from c_p(T_inf) = c_p,inf; Pr from Sutherland's and Keyes' laws
    if (!(c.gamma > 1.0) || !(c.Re > 0.0)) { delete ctx; return HRX_EINVAL; }
    const double a = (c.gamma - 1.0) / c.gamma, cp = TPG_R / a;
    ref.gamma = c.gamma; ref.Re = c.Re; ref.Ec = 1.0;
    ref.T_ref = (c.gamma - 1.0) * c.T_inf;
    ref.mu_inf = sutherland<double>(c.T_inf);
    ref.kappa_inf = keyes(c.T_inf);
    ref.Pr = ref.mu_inf * cp / ref.kappa_inf;
    ref.R_inf = TPG_R;
    d.tpg_k0 = 1.0 / (1.0 + a * tpg_vib(TPG_THETA / c.T_inf));
    d.tpg_th = TPG_THETA / ref.T_ref;
  } else {
    double Y[NS], ysum = 0.0;
    for (int s = 0; s < NS; ++s) { Y[s] = c.Y_inf[s]; ysum += Y[s]; }
    if (!(c.p_inf > 0.0) || fabs(ysum - 1.0) > 1e-9) { delete ctx; return HRX_EINVAL; }
    const double R = mixture_R(Y);
    SpeciesThermo st;
    species_e_cv(c.T_inf, st);
    double cv = 0.0;
    for (int s = 0; s < NS; ++s) cv += Y[s] * st.cv[s];
    const double cp = cv + R, g = cp / cv;
    const double rho = c.p_inf / (R * c.T_inf);
    const double cs = sqrt(g * R * c.T_inf);
    double X[NS], nsum = 0.0;
    for (int s = 0; s < NS; ++s) { X[s] = Y[s] / molar_mass(s); nsum += X[s]; }
    for (int s = 0; s < NS; ++s) X[s] = X[s] / nsum;
    Transport<double> tr;
    mixture_transport<double>(c.T_inf, c.p_inf, X, st.cv, tr);
    double L = c.L_ref, Re = c.Re;
    if (L > 0.0) Re = rho * cs * L / tr.mu;
    else {
      if (!(Re > 0.0)) { delete ctx; return HRX_EINVAL; }
      L = Re * tr.mu / (rho * cs);
    }
    ref.gamma = g; ref.Re = Re; ref.Pr = tr.mu * cp / tr.kappa;
    ref.T_ref = (g - 1.0) * c.T_inf; ref.Ec = cs * cs / (cp * ref.T_ref);
    ref.rho_inf = rho; ref.c_inf = cs; ref.mu_inf = tr.mu; ref.kappa_inf = tr.kappa;
    ref.R_inf = R; ref.L_ref = L;
  }
  d.gamma = ref.gamma; d.Re = ref.Re; d.Pr = ref.Pr; d.T_ref = ref.T_ref;
  d.mu_inf = ref.mu_inf; d.kappa_inf = ref.kappa_inf; d.c_inf = ref.c_inf;
  d.rho_inf = ref.rho_inf; d.L_ref = ref.L_ref; d.R_inf = ref.R_inf;
  d.iT_ref = 1.0 / d.T_ref;
  d.ic2 = 1.0 / (d.c_inf * d.c_inf);
  d.p_fac = (d.gamma - 1.0) / (d.gamma * d.R_inf);
  d.imu_inf = 1.0 / d.mu_inf;
  d.ikappa_inf = 1.0 / d.kappa_inf;
  d.iDscale = 1.0 / (d.c_inf * d.L_ref);
  d.wscale = d.L_ref / (d.rho_inf * d.c_inf);
  d.ic_inf = 1.0 / d.c_inf;
  // ---------------------------------------------------------- metrics, spacing, sponge
  std::vector<double> x(c.x, c.x + c.nx), y(c.y, c.y + c.ny), Dx, Dy, Dx6, Dy6;
  const bool compact = c.fd_scheme == HRX_FD_COMPACT;
  HostCLine cl[3];
  if (compact) {
    // metrics d(xi)/dx = 1 / (D x) with the compact operator itself
    cl[0] = compact_factors(c.nx, c.fd_order, false);
    cl[1] = compact_factors(c.ny, c.fd_order, false);
    if (c.nz > 1) cl[2] = compact_factors(c.nz, c.fd_order, true);
    host_compact_deriv(x, c.fd_order, cl[0], Dx);
    host_compact_deriv(y, c.fd_order, cl[1], Dy);
  } else {
    host_deriv(x, c.fd_order, Dx);
    host_deriv(y, c.fd_order, Dy);
  }
  host_deriv(x, 6, Dx6);
  host_deriv(y, 6, Dy6);
  const int nz = c.nz;
  std::vector<double> hm(2 * c.nx + 2 * c.ny + 2 * nz + c.nx + c.ny + nz, 0.0);
  double* mx = hm.data();
  double* sxv = mx + c.nx;
  double* dlx = sxv + c.nx;
  double* my = dlx + c.nx;
  double* syv = my + c.ny;
  double* dly = syv + c.ny;
  double* mz = dly + c.ny;
  double* dlz = mz + nz;
  for (int i = 0; i < c.nx; ++i) {
    mx[i] = 1.0 / Dx[i];
    if (!(Dx[i] > 0.0)) { delete ctx; return HRX_EINVAL; }
    dlx[i] = 1.0 / (1.0 / Dx6[i]);
  }
  for (int j = 0; j < c.ny; ++j) {
    my[j] = 1.0 / Dy[j];
    if (!(Dy[j] > 0.0)) { delete ctx; return HRX_EINVAL; }
    dly[j] = 1.0 / (1.0 / Dy6[j]);
  }
  for (int k = 0; k < nz; ++k) {
    if (nz > 1) {
      const double dz = c.z[1] - c.z[0];
      mz[k] = 1.0 / dz;
      dlz[k] = dz;
    } else {
      mz[k] = 0.0;
      dlz[k] = 1.0;
    }
  }
  // sponge: sigma_max s^3 with s the normalised depth (Eq. 26, cubic profile)
  if (c.sponge_in > 0) {
    const int i1 = c.sponge_in;
    for (int i = 0; i < i1; ++i) {
      const double s = (x[i1] - x[i]) / (x[i1] - x[0]);
      sxv[i] = fmax(sxv[i], c.sigma_max * (s * s * s));
    }
  }
  if (c.sponge_out > 0) {
    const int i0 = c.nx - 1 - c.sponge_out;
    for (int i = i0 + 1; i < c.nx; ++i) {
      const double s = (x[i] - x[i0]) / (x[c.nx - 1] - x[i0]);
      sxv[i] = fmax(sxv[i], c.sigma_max * (s * s * s));
    }
  }
  if (c.sponge_top > 0) {
    const int j0 = c.ny - 1 - c.sponge_top;
    for (int j = j0 + 1; j < c.ny; ++j) {
      const double s = (y[j] - y[j0]) / (y[c.ny - 1] - y[j0]);
      syv[j] = fmax(syv[j], c.sigma_max * (s * s * s));
    }
  }
  int rc = HRX_OK;
  auto fail = [&](int code) { hrx_destroy(ctx); return code; };
  if (hipMalloc(&ctx->metrics, hm.size() * sizeof(double)) != hipSuccess) return fail(HRX_ENOMEM);
  if ((rc = check(hipMemcpy(ctx->metrics, hm.data(), hm.size() * sizeof(double),
                            hipMemcpyHostToDevice))))
    return fail(rc);
  double* dm = ctx->metrics;
  d.mx = dm; d.sx = dm + c.nx; d.dlx = dm + 2 * c.nx;
  d.my = dm + 3 * c.nx; d.sy = d.my + c.ny; d.dly = d.my + 2 * c.ny;
  d.mz = d.my + 3 * c.ny; d.dlz = d.mz + nz;
  if (c.n_hold > 0) {
    std::vector<unsigned char> hm8((size_t)nz * 3 * c.nx, 0);
    for (int64_t h = 0; h < c.n_hold; ++h) {
      const long q = c.hold[h];
      const int i = (int)(q % c.nx);
      const long r = q / c.nx;
      const int j = (int)(r % c.ny);
      const int k = (int)(r / c.ny);
      hm8[((size_t)k * 3 + j) * c.nx + i] = 1;
    }
    if (hipMalloc(&ctx->hold, hm8.size()) != hipSuccess) return fail(HRX_ENOMEM);
    if ((rc = check(hipMemcpy(ctx->hold, hm8.data(), hm8.size(), hipMemcpyHostToDevice))))
      return fail(rc);
    d.hold = ctx->hold;
  }
  // ---------------------------------------------------------- scratch planes
  d.nsrc = nd + 1 + (c.gas == HRX_GAS_AIR5 ? NS : 0);
  d.w_p = d.nsrc;
  ctx->nWd = d.nsrc + 1;
  int w = 0;
  d.w_mu = w++;
  if (c.gas == HRX_GAS_AIR5) {
    d.w_kap = w++;
    d.w_D = w; w += NS;
    d.w_wdot = w; w += NS;
    if (c.diffusion == HRX_DIFF_STEFAN_MAXWELL) {
      d.sm = 1;
      d.w_iD = w; w += 10;
    }
  } else if (c.gas == HRX_GAS_TPG) {
    d.w_kap = w++;
  }
  if (d.ad_on) d.w_c = w++;
  ctx->nWp = w;
  ctx->nF = nd * d.nvar;
  d.nad = 3 + (c.gas == HRX_GAS_AIR5 ? NS : 0);
  const size_t rts = c.precision == HRX_PREC_MIXED ? sizeof(float) : sizeof(double);
  ctx->rt_size = rts;
  if (hipMalloc(&ctx->Wd, sizeof(double) * N * ctx->nWd) != hipSuccess) return fail(HRX_ENOMEM);
  if (hipMalloc(&ctx->Wp, rts * N * ctx->nWp) != hipSuccess) return fail(HRX_ENOMEM);
  if (hipMalloc(&ctx->F, sizeof(double) * N * ctx->nF) != hipSuccess) return fail(HRX_ENOMEM);
  if (hipMalloc(&ctx->R, sizeof(double) * N * d.nvar) != hipSuccess) return fail(HRX_ENOMEM);
  if (d.ad_on && hipMalloc(&ctx->AD, rts * N * d.nad * 2) != hipSuccess) return fail(HRX_ENOMEM);
  d.ad = ctx->AD;
  if (compact) {
    // factors of the three directions: [lo, up, iu] per direction, then q of z
    const int nzc = c.nz > 1 ? c.nz : 0;
    std::vector<double> hc;
    for (int a = 0; a < 3; ++a)
      for (const std::vector<double>* v : {&cl[a].lo, &cl[a].up, &cl[a].iu})
        hc.insert(hc.end(), v->begin(), v->end());
    if (nzc) hc.insert(hc.end(), cl[2].q.begin(), cl[2].q.end());
    if (hipMalloc(&ctx->cmat, hc.size() * sizeof(double)) != hipSuccess) return fail(HRX_ENOMEM);
    if ((rc = check(hipMemcpy(ctx->cmat, hc.data(), hc.size() * sizeof(double),
                              hipMemcpyHostToDevice))))
      return fail(rc);
    const double* q = ctx->cmat;
    for (int a = 0; a < 3; ++a) {
      const size_t n = cl[a].lo.size();
      d.cl[a].lo = q; d.cl[a].up = q + n; d.cl[a].iu = q + 2 * n;
      q += 3 * n;
      d.cl[a].s = cl[a].s;
      d.cl[a].alpha = cl[a].alpha;
    }
    d.cl[2].q = nzc ? q : nullptr;
    d.compact = 1;
    if (hipMalloc(&ctx->G, sizeof(double) * N * nd * d.nsrc) != hipSuccess) return fail(HRX_ENOMEM);
    if (cd_needs_temp(d) && hipMalloc(&ctx->Ct, sizeof(double) * N * d.nvar) != hipSuccess)
      return fail(HRX_ENOMEM);
  }
  if (hipMalloc(&ctx->counters, NCOUNT * CSLOTS * sizeof(unsigned long long)) != hipSuccess)
    return fail(HRX_ENOMEM);
  if ((rc = check(hipMemset(ctx->counters, 0, NCOUNT * CSLOTS * sizeof(unsigned long long)))))
    return fail(rc);
  d.counters = ctx->counters;
  {
    int dev = 0, ncu = 0;
    if ((rc = check(hipGetDevice(&dev)))) return fail(rc);
    if ((rc = check(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev))))
      return fail(rc);
    ctx->small_grid = (long)N <= 2L * 64 * 4 * ncu;   // 4 SIMDs per compute unit
    // the static workspace of hrx_rhs_eval_noalloc on this device (looked up once per
    // device; a failure only disables that entry point)
    if (scratch_address(dev, &ctx->noalloc) != HRX_OK) ctx->noalloc = nullptr;
  }
  // zeroed temperature plane: the first energy inversion starts cold
  if ((rc = check(hipMemset(ctx->Wd, 0, sizeof(double) * N * ctx->nWd)))) return fail(rc);
  *out = ctx;
  return HRX_OK;
}

int hrx_get_reference(const hrx_ctx* ctx, hrx_reference* out) {
  if (!ctx || !out) return HRX_EINVAL;
  *out = ctx->ref;
  return HRX_OK;
}

}  // extern "C"

namespace {

template <int GAS, int ND, int ORDER, bool AD, class RT>
void launch_flux(hrx_ctx* ctx, hipStream_t st, const double* Q, const double* Wd, const RT* Wp,
                 const RT* Gad, double* F) {
  const Dev& d = ctx->dev;
  constexpr int NSRC = ND + 1 + (GAS == AIR5 ? NS : 0);
  const unsigned nt = ND == 2 ? (unsigned)d.tgx * d.tgy : (unsigned)(d.tgx * d.tgz * d.ny);
  const size_t sh = NSRC * TILE_E * sizeof(double);
  timed(ctx, K_FLUX, st, [&] {
    if constexpr (GAS == AIR5) {
      if (d.sm) {   // Stefan-Maxwell diffusion
        if (ND == 2 && ctx->small_grid && sizeof(RT) == sizeof(double))
          k_flux_small<GAS, ND, ORDER, AD, RT, true><<<nt, TTX * TTY, sh, st>>>(d, Q, Wd, Wp,
                                                                                Gad, F);
        else
          k_flux<GAS, ND, ORDER, AD, RT, true><<<nt, TTX * TTY, sh, st>>>(d, Q, Wd, Wp, Gad, F);
        return;
      }
    }
    if constexpr (ND == 2 && sizeof(RT) == sizeof(double)) {
      if (ctx->small_grid) {
        k_flux_small<GAS, ND, ORDER, AD, RT><<<nt, TTX * TTY, sh, st>>>(d, Q, Wd, Wp, Gad, F);
        return;
      }
    }
    k_flux<GAS, ND, ORDER, AD, RT><<<nt, TTX * TTY, sh, st>>>(d, Q, Wd, Wp, Gad, F);
  });
}

// Grids up to this many points run the component chunks of a tile side by side in k_div
// (near two wavefronts per SIMD the chunks of a tile are latency bound).
constexpr long DIV_SPLIT_MAX_POINTS = 1L << 18;
// 3-D RK stages: the y march (k_div3m) instead of one row per block
constexpr bool DIV_MARCH3 = true;

template <int GAS, int ND, int ORDER, int MODE, class RT>
void launch_div(hrx_ctx* ctx, hipStream_t st, const double* F, const RT* Wp, const double* Q,
                const double* Qref, double* R, double* Qio, double* dQ, double A, double B,
                double dt, int rkf) {
  const Dev& d = ctx->dev;
  constexpr int nvar = (GAS == AIR5 ? NS : 1) + ND + 1;
  unsigned nt = ND == 2 ? (unsigned)d.tgx * d.tgy : (unsigned)(d.tgx * d.tgz * d.ny);
  constexpr int KC = div_chunk(ND);
  constexpr int nch = (nvar + KC - 1) / KC;
  const bool split = d.N <= DIV_SPLIT_MAX_POINTS;
  const size_t sh = (size_t)KC * (FXE + FYE) * sizeof(double);
  timed(ctx, K_DIV, st, [&] {
    if constexpr (ND == 2 && nch == 2) {
      // small grids: the two chunks of a tile in two halves of one 512-thread block;
      // larger grids: one block runs both chunks, the first one's inputs preloaded
      if (split)
        k_div<GAS, ND, ORDER, MODE, RT, false, 2>
            <<<nt, 2 * TTX * TTY, 2 * sh, st>>>(d, F, Wp, Q, Qref, R, Qio, dQ, A, B, dt, rkf);
      else
        k_div<GAS, ND, ORDER, MODE, RT, true, 1>
            <<<nt, TTX * TTY, sh, st>>>(d, F, Wp, Q, Qref, R, Qio, dQ, A, B, dt, rkf);
      return;
    }
    if constexpr (ND == 3 && MODE == MODE_RK) {
      if (DIV_MARCH3) {
        // march along y in segments of rseg rows (shorter on small grids, for more blocks)
        const int rseg = d.N >= (1L << 22) ? 32 : 8;
        const int nseg = (d.ny + rseg - 1) / rseg;
        constexpr int nchm = (nvar + KCM - 1) / KCM;
        const size_t shm = (size_t)2 * KCM * (FXE + FYE) * sizeof(double);
        k_div3m<GAS, ORDER, RT><<<(unsigned)(d.tgx * d.tgz * nseg * nchm), TTX * TTY, shm, st>>>(
            d, F, Wp, Qref, Qio, dQ, A, B, dt, rkf, rseg, nseg);
        return;
      }
    }
    k_div<GAS, ND, ORDER, MODE, RT, false, 1>
        <<<split ? nt * nch : nt, TTX * TTY, sh, st>>>(d, F, Wp, Q, Qref, R, Qio, dQ, A, B, dt,
                                                         rkf);
  });
}

// The pointwise pass (and in the surrogate form the network pass before it)
template <int GAS, int ND, class RT>
void launch_prim(hrx_ctx* ctx, const double* Q, hipStream_t st) {
  const Dev& d = ctx->dev;
  const long N = d.N;
  const int bs = 128;
  const unsigned nb = blocks_for(N, bs);
  double* Wd = ctx->Wd;
  RT* Wp = (RT*)ctx->Wp;
  if (GAS == AIR5 && ctx->thermo_mode == HRX_THERMO_SURROGATE) {
    // network pass (its outputs in the context's ys workspace), then the pointwise pass
    const unsigned nbs = (unsigned)std::min<long>((N + 255) / 256, 2048);
    timed(ctx, K_PRIM, st, [&] {
      k_mlp_eval<ND, true><<<nbs, 256, 0, st>>>(d, ctx->norm_dev, N, N, nullptr, nullptr, nullptr, Q,
                                                ctx->ys, ctx->wsw, ctx->bias);
      k_prim<GAS, ND, RT, true><<<nb, bs, 0, st>>>(d, Q, Wd, Wp, ctx->ys);
    });
  } else {
    timed(ctx, K_PRIM, st, [&] { k_prim<GAS, ND, RT><<<nb, bs, 0, st>>>(d, Q, Wd, Wp, nullptr); });
  }
}

// The artificial-diffusivity smoothing passes after the sources: fourth differences with
// the x and y filters, and (3-D) the z filter; returns the planes the flux reads.
template <int GAS, int ND, class RT>
const RT* launch_ad_smoothing(hrx_ctx* ctx, hipStream_t st, bool zpass = true) {
  const Dev& d = ctx->dev;
  const long N = d.N;
  RT* A = (RT*)ctx->AD;
  RT* B = A + (long)d.nad * N;
  timed(ctx, K_AD_D4, st, [&] {
    const int mseg = ND == 2 ? MSEG2 : MSEG3;
    const int nstrip = (d.nx + MO - 1) / MO, nseg = (d.ny + mseg - 1) / mseg;
    if constexpr (ND == 3) {
      constexpr int NWZ = AD_MARCH_NWZ;
      const int nzg = (d.nz + NWZ - 1) / NWZ;
      k_ad_march3<GAS, RT, NWZ, AD_MARCH_PD><<<(unsigned)((long)nzg * nstrip * nseg * d.nad),
                                               MW * NWZ, 0, st>>>(d, A, B, nstrip, nseg, mseg,
                                                                 nzg);
    } else {
      k_ad_march<GAS, RT><<<(unsigned)((long)nstrip * nseg * d.nad), MW, 0, st>>>(
          d, A, B, nstrip, nseg, mseg);
    }
  });
  if (ND == 3 && zpass) {
    const int nxs = (d.nx + 63) / 64, nzs = (d.nz + ZSEG - 1) / ZSEG;
    timed(ctx, K_AD_FZ, st, [&] {
      k_ad_filter_z<RT><<<(unsigned)((long)nxs * d.ny * nzs * d.nad), 64, 0, st>>>(d, B, A, nxs,
                                                                                nzs);
    });
    return A;
  }
  return B;
}

template <int GAS, int ND, int ORDER, class RT>
int launch_rhs_chain(hrx_ctx* ctx, const double* Q, hipStream_t st) {
  const Dev& d = ctx->dev;
  double* Wd = ctx->Wd;
  RT* Wp = (RT*)ctx->Wp;
  double* F = ctx->F;
  launch_prim<GAS, ND, RT>(ctx, Q, st);
  if (d.ad_on) {
    const unsigned nts = ND == 2 ? (unsigned)d.tgx * d.tgy : (unsigned)(d.tgx * d.tgz * d.ny);
    timed(ctx, K_AD_SRC, st, [&] {
      if constexpr (ND == 3) {
        const int rseg = d.N >= (1L << 22) ? 32 : 8;
        const int nseg = (d.ny + rseg - 1) / rseg;
        k_ad_src3m<ORDER, RT><<<(unsigned)(d.tgx * d.tgz * nseg), TTX * TTY,
                                 2 * ND * TILE_E * sizeof(double), st>>>(d, Wd, (RT*)ctx->AD,
                                                                         rseg, nseg);
      } else {
        k_ad_src<GAS, ND, ORDER, RT><<<nts, TTX * TTY, ND * TILE_E * sizeof(double), st>>>(
            d, Wd, (RT*)ctx->AD);
      }
    });
    // 3-D: the flux applies the z filter itself (FLUX_ZFILTER)
    const RT* Gad = launch_ad_smoothing<GAS, ND, RT>(ctx, st, !(ND == 3 && FLUX_ZFILTER));
    launch_flux<GAS, ND, ORDER, true, RT>(ctx, st, Q, Wd, Wp, Gad, F);
  } else {
    launch_flux<GAS, ND, ORDER, false, RT>(ctx, st, Q, Wd, Wp, nullptr, F);
  }
  return check(hipGetLastError());
}

// Wall-row pass after an unfused update (every gas and dimension)
void launch_bc(hrx_ctx* ctx, double* Q, hipStream_t st) {
  const Dev& d = ctx->dev;
  const long nw = (long)(d.nx - 1) * d.nz;
  const unsigned nb = blocks_for(nw, 128);
  const bool air = ctx->cfg.gas == HRX_GAS_AIR5, tpg = ctx->cfg.gas == HRX_GAS_TPG;
  timed(ctx, K_BC, st, [&] {
    if (d.ndim == 2) {
      if (air) k_bc<AIR5, 2><<<nb, 128, 0, st>>>(d, Q);
      else if (tpg) k_bc<TPG, 2><<<nb, 128, 0, st>>>(d, Q);
      else k_bc<CPG, 2><<<nb, 128, 0, st>>>(d, Q);
    } else {
      if (air) k_bc<AIR5, 3><<<nb, 128, 0, st>>>(d, Q);
      else if (tpg) k_bc<TPG, 3><<<nb, 128, 0, st>>>(d, Q);
      else k_bc<CPG, 3><<<nb, 128, 0, st>>>(d, Q);
    }
  });
}

// Compact first derivatives of nplanes planes along direction dir: f (plane stride fps)
// -> out (plane stride ops), out = scale m D f, or out += scale m D f (acc; the forward
// values then go through the context's temporary planes).
void launch_cd(hrx_ctx* ctx, int dir, const double* f, long fps, double* out, long ops,
               int nplanes, bool acc, double scale, hipStream_t st) {
  const Dev& d = ctx->dev;
  const long N = d.N;
  const int ord = d.fd_order;
  timed(ctx, K_CDERIV, st, [&] {
    if (dir == 0) {
      // chunks of C = the power of two >= nx / 64 points per lane, four wavefronts per
      // block within 64 KB of LDS (factors + one array per wavefront)
      const long nlines = N / d.nx;
      int C = 1;
      while (64 * C < d.nx) C *= 2;
      const long S = 64L * C;
      const int nw = (int)std::max(1L, std::min(4L, (65536L / (8 * S)) - 3));
      // K lines per wavefront (up to 8) while the launch keeps 2048 or more blocks
      int K = 1;
      while (K < 8 && nlines * nplanes >= (long)nw * (2 * K) * 2048) K *= 2;
      const dim3 g((unsigned)((nlines + (long)nw * K - 1) / ((long)nw * K)), (unsigned)nplanes);
      const size_t sh = (size_t)(3 + nw) * S * sizeof(double);
      auto go = [&](auto cc) {
        constexpr int CC = decltype(cc)::value;
        auto gk = [&](auto kk) {
          constexpr int KK = decltype(kk)::value;
          if (acc)
            k_cd_xp<true, CC, KK><<<g, 64 * nw, sh, st>>>(d.nx, nlines, f, fps, out, ops, d.mx,
                                                           scale, ord, d.cl[0]);
          else
            k_cd_xp<false, CC, KK><<<g, 64 * nw, sh, st>>>(d.nx, nlines, f, fps, out, ops, d.mx,
                                                            scale, ord, d.cl[0]);
        };
        switch (K) {
          case 1: gk(std::integral_constant<int, 1>()); break;
          case 2: gk(std::integral_constant<int, 2>()); break;
          case 4: gk(std::integral_constant<int, 4>()); break;
          default: gk(std::integral_constant<int, 8>()); break;
        }
      };
      switch (C) {
        case 1: go(std::integral_constant<int, 1>()); break;
        case 2: go(std::integral_constant<int, 2>()); break;
        case 4: go(std::integral_constant<int, 4>()); break;
        case 8: go(std::integral_constant<int, 8>()); break;
        case 16: go(std::integral_constant<int, 16>()); break;
        default: {
          // longer lines (C = 32 would need 80 KB of LDS per line): one wavefront per line
          // with the line in LDS by point
          const dim3 g1((unsigned)nlines, (unsigned)nplanes);
          const size_t sh1 = 2 * (size_t)d.nx * sizeof(double);
          if (acc)
            k_cd_x<true><<<g1, 64, sh1, st>>>(d.nx, f, fps, out, ops, d.mx, scale, ord, d.cl[0]);
          else
            k_cd_x<false><<<g1, 64, sh1, st>>>(d.nx, f, fps, out, ops, d.mx, scale, ord, d.cl[0]);
        }
      }
    } else if (cdcol_fits(dir == 1 ? d.ny : d.nz)) {
      // lines of up to 512 points: 16 lines per block, held on chip (k_cd_colp)
      const bool yl = dir == 1;
      const int n = yl ? d.ny : d.nz;
      const long s = yl ? (long)d.nx : (long)d.nx * d.ny;
      const long s2 = yl ? (long)d.nx * d.ny : (long)d.nx;
      const long nc2 = yl ? d.nz : d.ny;
      const int CL = cdcol_chunk(n);
      const dim3 g((unsigned)(((d.nx + 15) / 16) * nc2), (unsigned)nplanes);
      const size_t sh = (size_t)(256 + 16 * (yl ? 3 : 4)) * CL * sizeof(double);
      const double* mm = yl ? d.my : d.mz;
      const CLine& cl = d.cl[dir];
      auto go = [&](auto cc) {
        constexpr int CC = decltype(cc)::value;
        if (yl) {
          if (acc) k_cd_colp<true, false, CC><<<g, 256, sh, st>>>(n, s, d.nx, s2, f, fps, out, ops, mm, scale, ord, cl);
          else k_cd_colp<false, false, CC><<<g, 256, sh, st>>>(n, s, d.nx, s2, f, fps, out, ops, mm, scale, ord, cl);
        } else {
          if (acc) k_cd_colp<true, true, CC><<<g, 256, sh, st>>>(n, s, d.nx, s2, f, fps, out, ops, mm, scale, ord, cl);
          else k_cd_colp<false, true, CC><<<g, 256, sh, st>>>(n, s, d.nx, s2, f, fps, out, ops, mm, scale, ord, cl);
        }
      };
      switch (CL) {
        case 1: go(std::integral_constant<int, 1>()); break;
        case 2: go(std::integral_constant<int, 2>()); break;
        case 4: go(std::integral_constant<int, 4>()); break;
        case 8: go(std::integral_constant<int, 8>()); break;
        case 16: go(std::integral_constant<int, 16>()); break;
        default: go(std::integral_constant<int, 32>()); break;
      }
    } else if (dir == 1) {
      const dim3 g(blocks_for((long)d.nx * d.nz, 128), (unsigned)nplanes);
      const long s2 = (long)d.nx * d.ny;
      if (acc)
        k_cd_col<true, false><<<g, 128, 0, st>>>(d.ny, d.nx, d.nx, d.nz, s2, f, fps, out, ops,
                                                ctx->Ct, N, d.my, scale, ord, d.cl[1]);
      else
        k_cd_col<false, false><<<g, 128, 0, st>>>(d.ny, d.nx, d.nx, d.nz, s2, f, fps, out, ops,
                                                 ctx->Ct, N, d.my, scale, ord, d.cl[1]);
    } else {
      const dim3 g(blocks_for((long)d.nx * d.ny, 128), (unsigned)nplanes);
      const long s = (long)d.nx * d.ny;
      if (acc)
        k_cd_col<true, true><<<g, 128, 0, st>>>(d.nz, s, d.nx, d.ny, d.nx, f, fps, out, ops,
                                               ctx->Ct, N, d.mz, scale, ord, d.cl[2]);
      else
        k_cd_col<false, true><<<g, 128, 0, st>>>(d.nz, s, d.nx, d.ny, d.nx, f, fps, out, ops,
                                                ctx->Ct, N, d.mz, scale, ord, d.cl[2]);
    }
  });
}

// One right-hand side (and stage) with compact first derivatives:
//   k_prim -> gradients of u, (v, w), T, (X_s) along every direction (line solves)
//   -> [artificial diffusivity: sources from the gradient planes, smoothing]
//   -> k_flux_c (fluxes from the gradient planes) -> divergence, -sum_j D_j F_j, by line
//   solves accumulating into Racc -> k_fin (sources, sponge, held rows, update)
//   -> wall pass (stages).
template <int GAS, int ND, class RT>
int run_compact(hrx_ctx* ctx, int mode, const double* Q, const double* Qref, double* R,
                double* Qio, double* dQ, double A, double B, double dt, int rkf, hipStream_t st) {
  const Dev& d = ctx->dev;
  const long N = d.N;
  constexpr int nvar = (GAS == AIR5 ? NS : 1) + ND + 1;
  const double* Qs = mode == MODE_RHS ? Q : Qio;
  double* Wd = ctx->Wd;
  RT* Wp = (RT*)ctx->Wp;
  double* F = ctx->F;
  double* G = ctx->G;
  const int nsrc = d.nsrc;
  launch_prim<GAS, ND, RT>(ctx, Qs, st);
  for (int b = 0; b < ND; ++b)
    launch_cd(ctx, b, Wd, N, G + (long)b * nsrc * N, N, nsrc, false, 1.0, st);
  const RT* Gad = nullptr;
  const unsigned nb = blocks_for(N, 256);
  if (d.ad_on) {
    timed(ctx, K_AD_SRC, st, [&] { k_ad_src_c<ND, RT><<<nb, 256, 0, st>>>(d, G, (RT*)ctx->AD); });
    Gad = launch_ad_smoothing<GAS, ND, RT>(ctx, st);
  }
  timed(ctx, K_FLUX, st, [&] {
    if constexpr (GAS == AIR5) {
      if (d.sm) {
        if (d.ad_on) k_flux_c<GAS, ND, true, RT, true><<<nb, 256, 0, st>>>(d, Qs, Wd, Wp, Gad, F, G);
        else k_flux_c<GAS, ND, false, RT, true><<<nb, 256, 0, st>>>(d, Qs, Wd, Wp, Gad, F, G);
        return;
      }
    }
    if (d.ad_on) k_flux_c<GAS, ND, true, RT><<<nb, 256, 0, st>>>(d, Qs, Wd, Wp, Gad, F, G);
    else k_flux_c<GAS, ND, false, RT><<<nb, 256, 0, st>>>(d, Qs, Wd, Wp, Gad, F, G);
  });
  double* Racc = mode == MODE_RHS ? R : ctx->R;
  for (int b = 0; b < ND; ++b)
    launch_cd(ctx, b, F + (long)b * nvar * N, N, Racc, N, nvar, b > 0, -1.0, st);
  timed(ctx, K_FIN, st, [&] {
    if (mode == MODE_RHS)
      k_fin<GAS, ND, MODE_RHS, RT><<<nb, 256, 0, st>>>(d, Wp, Q, Qref, Racc, R, nullptr, nullptr,
                                                      0.0, 0.0, 0.0, RKF_2N);
    else
      k_fin<GAS, ND, MODE_RK, RT><<<nb, 256, 0, st>>>(d, Wp, nullptr, Qref, Racc, nullptr, Qio, dQ,
                                                     A, B, dt, rkf);
  });
  if (mode == MODE_RK) launch_bc(ctx, Qio, st);
  ctx->dev.warm = 1;
  return check(hipGetLastError());
}

template <int GAS, int ND, int ORDER, class RT>
int run(hrx_ctx* ctx, int mode, const double* Q, const double* Qref, double* R, double* Qio,
        double* dQ, double A, double B, double dt, int rkf, hipStream_t st) {
  const Dev& d = ctx->dev;
  int rc = launch_rhs_chain<GAS, ND, ORDER, RT>(ctx, mode == MODE_RHS ? Q : Qio, st);
  if (rc) return rc;
  ctx->dev.warm = 1;
  const unsigned ng = (unsigned)d.gx * d.ny * d.nz;
  const double* F = ctx->F;
  const RT* Wp = (const RT*)ctx->Wp;
  if (mode == MODE_RHS) {
    launch_div<GAS, ND, ORDER, MODE_RHS, RT>(ctx, st, F, Wp, Q, Qref, R, nullptr, nullptr, 0.0,
                                             0.0, 0.0, RKF_2N);
  } else {
    launch_div<GAS, ND, ORDER, MODE_RK, RT>(ctx, st, F, Wp, nullptr, Qref, nullptr, Qio, dQ, A,
                                            B, dt, rkf);
    constexpr int nvar = (GAS == AIR5 ? NS : 1) + ND + 1;
    constexpr int nch = (nvar + div_chunk(ND) - 1) / div_chunk(ND);
    // chunks of one tile in separate blocks (two chunks share a block in 2-D)
    const bool split = d.N <= DIV_SPLIT_MAX_POINTS && nch > 2;
    if (ND == 3 || split) {   // else it ran inside k_div
      const long nw = (long)(d.nx - 1) * d.nz;
      timed(ctx, K_BC, st, [&] { k_bc<GAS, ND><<<blocks_for(nw, 128), 128, 0, st>>>(d, Qio); });
    }
  }
  return check(hipGetLastError());
}

int dispatch(hrx_ctx* ctx, int mode, const double* Q, const double* Qref, double* R, double* Qio,
             double* dQ, double A, double B, double dt, int rkf, hipStream_t st) {
  const Dev& d = ctx->dev;
  const bool air = ctx->cfg.gas == HRX_GAS_AIR5, tpg = ctx->cfg.gas == HRX_GAS_TPG;
  const bool o6 = d.fd_order == 6;
  const bool mixed = ctx->cfg.precision == HRX_PREC_MIXED;
  if (d.compact) {
#define HRX_RUNC(G, NDV)                                                                   \
  return mixed ? run_compact<G, NDV, float>(ctx, mode, Q, Qref, R, Qio, dQ, A, B, dt, rkf, st) \
               : run_compact<G, NDV, double>(ctx, mode, Q, Qref, R, Qio, dQ, A, B, dt, rkf, st)
    if (d.ndim == 2) {
      if (air) HRX_RUNC(AIR5, 2);
      else if (tpg) HRX_RUNC(TPG, 2);
      else HRX_RUNC(CPG, 2);
    } else {
      if (air) HRX_RUNC(AIR5, 3);
      else if (tpg) HRX_RUNC(TPG, 3);
      else HRX_RUNC(CPG, 3);
    }
#undef HRX_RUNC
  }
#define HRX_RUN(G, NDV, O)                                                              \
  return mixed ? run<G, NDV, O, float>(ctx, mode, Q, Qref, R, Qio, dQ, A, B, dt, rkf, st) \
               : run<G, NDV, O, double>(ctx, mode, Q, Qref, R, Qio, dQ, A, B, dt, rkf, st)
  if (d.ndim == 2) {
    if (air) { if (o6) HRX_RUN(AIR5, 2, 6); else HRX_RUN(AIR5, 2, 4); }
    else if (tpg) { if (o6) HRX_RUN(TPG, 2, 6); else HRX_RUN(TPG, 2, 4); }
    else { if (o6) HRX_RUN(CPG, 2, 6); else HRX_RUN(CPG, 2, 4); }
  } else {
    if (air) { if (o6) HRX_RUN(AIR5, 3, 6); else HRX_RUN(AIR5, 3, 4); }
    else if (tpg) { if (o6) HRX_RUN(TPG, 3, 6); else HRX_RUN(TPG, 3, 4); }
    else { if (o6) HRX_RUN(CPG, 3, 6); else HRX_RUN(CPG, 3, 4); }
  }
#undef HRX_RUN
}

// Williamson 2N-RK3 and Carpenter-Kennedy 2N-RK4(3)5 coefficients
const double RK3A[3] = {0.0, -5.0 / 9.0, -153.0 / 128.0};
const double RK3B[3] = {1.0 / 3.0, 15.0 / 16.0, 8.0 / 15.0};
const double RK4A[5] = {0.0, -567301805773.0 / 1357537059087.0,
                        -2404267990393.0 / 2016746695238.0, -3550918686646.0 / 2091501179385.0,
                        -1275806237668.0 / 842570457699.0};
const double RK4B[5] = {1432997174477.0 / 9575080441755.0, 5161836677717.0 / 13612068292357.0,
                        1720146321549.0 / 2090206949498.0, 3134564353537.0 / 4481467310338.0,
                        2277821191437.0 / 14882151754819.0};
// Shu-Osher TVD RK3 as Q <- a_k Q0 + b_k (Q + dt R(Q))
const double SSPA[3] = {0.0, 3.0 / 4.0, 1.0 / 3.0};
const double SSPB[3] = {1.0, 1.0 / 4.0, 2.0 / 3.0};


}  // namespace

extern "C" {

int hrx_rhs_eval(hrx_ctx* ctx, const double* Q, const double* Q_ref, double* R,
                 void* hip_stream) {
  if (!ctx || !Q || !R || R == Q) return HRX_EINVAL;
  hipStream_t st = (hipStream_t)hip_stream;
  ctx->last_stream = st;
  return dispatch(ctx, MODE_RHS, Q, Q_ref, R, nullptr, nullptr, 0.0, 0.0, 0.0, RKF_2N, st);
}

int hrx_rhs_eval_noalloc(hrx_ctx* ctx, const double* Q, const double* Q_ref, double* R,
                         void* hip_stream) {
  if (!ctx || !Q || !R || R == Q) return HRX_EINVAL;
  // the surrogate form's network outputs are not part of the static layout
  if (ctx->thermo_mode == HRX_THERMO_SURROGATE) return HRX_EUNSUP;
  if (!ctx->noalloc) return HRX_EHIP;
  const Dev& d = ctx->dev;
  const size_t N = (size_t)d.N;
  auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
  const size_t bWd = al(sizeof(double) * N * ctx->nWd);
  const size_t bWp = al(ctx->rt_size * N * ctx->nWp);
  const size_t bF = al(sizeof(double) * N * ctx->nF);
  const size_t bAD = d.ad_on ? al(ctx->rt_size * N * d.nad * 2) : 0;
  const size_t bG = d.compact ? al(sizeof(double) * N * d.ndim * d.nsrc) : 0;
  const size_t bCt = cd_needs_temp(d) ? al(sizeof(double) * N * d.nvar) : 0;
  if (bWd + bWp + bF + bAD + bG + bCt > NOALLOC_BYTES) return HRX_ETOOBIG;
  hipStream_t st = (hipStream_t)hip_stream;
  ctx->last_stream = st;
  // The launches of this call take the static workspace in place of the context's
  // scratch (the pointers are passed to the kernels by value at launch); the energy
  // inversion starts cold, since the workspace holds whatever the last call left.
  unsigned char* base = static_cast<unsigned char*>(ctx->noalloc);
  double* const Wd0 = ctx->Wd;
  void* const Wp0 = ctx->Wp;
  double* const F0 = ctx->F;
  void* const AD0 = ctx->AD;
  double* const G0 = ctx->G;
  double* const Ct0 = ctx->Ct;
  const Dev dev0 = ctx->dev;
  ctx->Wd = reinterpret_cast<double*>(base);
  ctx->Wp = base + bWd;
  ctx->F = reinterpret_cast<double*>(base + bWd + bWp);
  ctx->AD = bAD ? base + bWd + bWp + bF : nullptr;
  ctx->G = bG ? reinterpret_cast<double*>(base + bWd + bWp + bF + bAD) : nullptr;
  ctx->Ct = bCt ? reinterpret_cast<double*>(base + bWd + bWp + bF + bAD + bG) : nullptr;
  ctx->dev.ad = ctx->AD;
  ctx->dev.warm = 0;
  const int rc = dispatch(ctx, MODE_RHS, Q, Q_ref, R, nullptr, nullptr, 0.0, 0.0, 0.0, RKF_2N, st);
  ctx->Wd = Wd0;
  ctx->Wp = Wp0;
  ctx->F = F0;
  ctx->AD = AD0;
  ctx->G = G0;
  ctx->Ct = Ct0;
  ctx->dev = dev0;
  return rc;
}

int hrx_rk_stage(hrx_ctx* ctx, int stage, double dt, double* Q, double* dQ, const double* Q_ref,
                 const double* R, void* hip_stream) {
  if (!ctx || !Q || !dQ || Q == dQ || stage < 0 || !std::isfinite(dt)) return HRX_EINVAL;
  if (R && (R == Q || R == dQ)) return HRX_EINVAL;
  const int sch = ctx->cfg.rk_scheme;
  const int ns = sch == HRX_RK45_2N ? 5 : 3;
  const int k = stage % ns;
  double A, B;
  int rkf = RKF_2N;
  if (sch == HRX_RK3_2N) {
    A = RK3A[k];
    B = RK3B[k];
  } else if (sch == HRX_RK45_2N) {
    A = RK4A[k];
    B = RK4B[k];
  } else {
    A = SSPA[k];
    B = SSPB[k];
    rkf = k == 0 ? RKF_SSP_FIRST : RKF_SSP;
  }
  hipStream_t st = (hipStream_t)hip_stream;
  ctx->last_stream = st;
  if (R) {
    // unfused: the caller's right-hand side, a pointwise update, the wall row
    const Dev& d = ctx->dev;
    timed(ctx, K_DIV, st, [&] {
      k_rk_update<<<blocks_for(d.N, 256), 256, 0, st>>>(d.N, d.nvar, R, Q, dQ, A, B, dt, rkf);
    });
    launch_bc(ctx, Q, st);
    return check(hipGetLastError());
  }
  // After the first stage (which switches the energy inversion to warm starts), a
  // stage's kernel sequence is captured once per argument set into a HIP graph and
  // replayed: one launch instead of four or more.  Not on the null stream (it cannot
  // be captured) and not while per-kernel timing is on.
  if (ctx->use_graphs && st != nullptr && !ctx->timing && ctx->dev.warm) {
    for (auto& g : ctx->graphs)
      if (g.Q == Q && g.dQ == dQ && g.Qref == Q_ref && g.dt == dt && g.k == k && g.st == st)
        return check(hipGraphLaunch(g.exec, st));
    if (ctx->graphs.size() >= 16) clear_graphs(ctx);
    if (hipStreamBeginCapture(st, hipStreamCaptureModeRelaxed) != hipSuccess) return HRX_EHIP;
    const int rc = dispatch(ctx, MODE_RK, nullptr, Q_ref, nullptr, Q, dQ, A, B, dt, rkf, st);
    hipGraph_t graph;
    if (hipStreamEndCapture(st, &graph) != hipSuccess || rc) return rc ? rc : HRX_EHIP;
    hipGraphExec_t exec;
    const hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ie != hipSuccess) return HRX_EHIP;
    ctx->graphs.push_back({Q, dQ, Q_ref, dt, k, st, exec});
    return check(hipGraphLaunch(exec, st));
  }
  return dispatch(ctx, MODE_RK, nullptr, Q_ref, nullptr, Q, dQ, A, B, dt, rkf, st);
}

int hrx_thermo_eval(hrx_ctx* ctx, int64_t n, const double* rho, const double* e, const double* Y,
                    double* T, double* p, double* h, double* mu, double* kappa, double* D,
                    int32_t* status, void* hip_stream) {
  if (!ctx || n < 0 || (n > 0 && (!rho || !e || !Y || !T))) return HRX_EINVAL;
  if (ctx->cfg.gas != HRX_GAS_AIR5) return HRX_EINVAL;
  if (n == 0) return HRX_OK;
  hipStream_t st = (hipStream_t)hip_stream;
  ctx->last_stream = st;
  const bool mixed = ctx->cfg.precision == HRX_PREC_MIXED;
  const bool sur = ctx->thermo_mode == HRX_THERMO_SURROGATE;
  if (sur && (!ctx->ys || ctx->ys_cap < 1)) return HRX_EINVAL;
  const double rt = ctx->dev.newton_rtol;
  const int mi = ctx->dev.newton_max;
  timed(ctx, K_THERMO, st, [&] {
    if (sur) {
      // the network's outputs for each chunk go through the workspace (no allocation)
      for (int64_t off = 0; off < n; off += ctx->ys_cap) {
        const int64_t m = std::min<int64_t>(ctx->ys_cap, n - off);
        auto at = [&](auto* a) { return a ? a + off : a; };
        const unsigned nbs = (unsigned)std::min<long>((m + 255) / 256, 2048);
        k_mlp_eval<2, false><<<nbs, 256, 0, st>>>(ctx->dev, ctx->norm_dev, m, n, rho + off,
                                                 e + off, Y + off, nullptr, ctx->ys, ctx->wsw,
                                                 ctx->bias);
        k_thermo_eval<double, true><<<blocks_for(m, 128), 128, 0, st>>>(
            m, n, rt, mi, rho + off, e + off, Y + off, T + off, at(p), at(h), at(mu), at(kappa),
            at(D), at(status), ctx->counters, ctx->ys);
      }
    } else if (mixed)
      k_thermo_eval<float><<<blocks_for(n, 128), 128, 0, st>>>(
          n, n, rt, mi, rho, e, Y, T, p, h, mu, kappa, D, status, ctx->counters, nullptr);
    else
      k_thermo_eval<double><<<blocks_for(n, 128), 128, 0, st>>>(
          n, n, rt, mi, rho, e, Y, T, p, h, mu, kappa, D, status, ctx->counters, nullptr);
  });
  return check(hipGetLastError());
}

int hrx_chem_source(hrx_ctx* ctx, int64_t n, const double* rho_s, const double* T, double* wdot,
                    void* hip_stream) {
  if (!ctx || n < 0 || (n > 0 && (!rho_s || !T || !wdot))) return HRX_EINVAL;
  if (ctx->cfg.gas != HRX_GAS_AIR5) return HRX_EINVAL;
  if (n == 0) return HRX_OK;
  hipStream_t st = (hipStream_t)hip_stream;
  ctx->last_stream = st;
  const bool mixed = ctx->cfg.precision == HRX_PREC_MIXED;
  timed(ctx, K_CHEM, st, [&] {
    if (mixed)
      k_chem_source<float><<<blocks_for(n, 128), 128, 0, st>>>(n, rho_s, T, wdot);
    else
      k_chem_source<double><<<blocks_for(n, 128), 128, 0, st>>>(n, rho_s, T, wdot);
  });
  return check(hipGetLastError());
}

int hrx_equilibrium(hrx_ctx* ctx, int64_t n, const double* rho, const double* T,
                    const double* xiN, double* Y, int32_t* status, void* hip_stream) {
  if (!ctx || n < 0 || (n > 0 && (!rho || !T || !Y))) return HRX_EINVAL;
  if (ctx->cfg.gas != HRX_GAS_AIR5) return HRX_EINVAL;
  if (n == 0) return HRX_OK;
  hipStream_t st = (hipStream_t)hip_stream;
  ctx->last_stream = st;
  const double* Yi = ctx->cfg.Y_inf;
  const double xi0 = Yi[0] + Yi[2] * (molar_mass(3) / molar_mass(2)) + Yi[3];
  timed(ctx, K_EQUIL, st, [&] {
    k_equilibrium<<<blocks_for(n, 128), 128, 0, st>>>(n, ctx->dev.newton_rtol, ctx->dev.newton_max,
                                                      rho, T, xiN, xi0, Y, status, ctx->counters);
  });
  return check(hipGetLastError());
}

int hrx_timing_enable(hrx_ctx* ctx, int on) {
  if (!ctx) return HRX_EINVAL;
  if (on) {
    if (!ctx->timing) {
      for (int i = 0; i < 8192; ++i) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return HRX_EHIP;
        ctx->ev_free.push_back(e);
      }
      for (int k = 0; k < HRX_NKERNELS; ++k) { ctx->ms[k] = 0.0; ctx->launches[k] = 0; }
      ctx->timing = true;
    }
    return HRX_OK;
  }
  int rc = flush_timing(ctx);
  for (auto e : ctx->ev_free) (void)hipEventDestroy(e);
  ctx->ev_free.clear();
  ctx->timing = false;
  return rc;
}

int hrx_timing_read(hrx_ctx* ctx, double* ms, int64_t* launches) {
  if (!ctx || !ms || !launches) return HRX_EINVAL;
  int rc = flush_timing(ctx);
  for (int k = 0; k < HRX_NKERNELS; ++k) { ms[k] = ctx->ms[k]; launches[k] = ctx->launches[k]; }
  return rc;
}

int hrx_get_counters(hrx_ctx* ctx, hrx_counters* out, int reset) {
  if (!ctx || !out) return HRX_EINVAL;
  std::vector<unsigned long long> hs((size_t)NCOUNT * CSLOTS);
  unsigned long long h[NCOUNT] = {0};
  int rc = check(hipStreamSynchronize(ctx->last_stream));
  if (rc) return rc;
  rc = check(hipMemcpy(hs.data(), ctx->counters, hs.size() * sizeof(unsigned long long),
                       hipMemcpyDeviceToHost));
  if (rc) return rc;
  for (int k = 0; k < NCOUNT; ++k)
    for (int q = 0; q < CSLOTS; ++q) h[k] += hs[(size_t)k * CSLOTS + q];
  out->newton_nonconverged = (int64_t)h[0];
  out->energy_below_min = (int64_t)h[1];
  out->surrogate_fallbacks = (int64_t)h[2];
  out->nonfinite = (int64_t)h[3];
  out->negative_density = (int64_t)h[4];
  if (reset) rc = check(hipMemset(ctx->counters, 0, hs.size() * sizeof(unsigned long long)));
  if (rc) return rc;
  if (h[3]) return HRX_ENONFINITE;
  if (h[1]) return HRX_EDOMAIN;
  if (h[0]) return HRX_ENEWTON;
  return HRX_OK;
}

}  // extern "C"

// ====================================================================== surrogate API
extern "C" {

int hrx_mlp_init(hrx_ctx* ctx, int64_t max_batch) {
  if (!ctx || max_batch < 1 || max_batch > (int64_t)1 << 24) return HRX_EINVAL;
  if (ctx->theta) return HRX_EINVAL;  // once per context
  const size_t P = MLP_NPARAM * sizeof(float);
  const size_t B = (size_t)max_batch;
  if (hipMalloc(&ctx->theta, P) != hipSuccess || hipMalloc(&ctx->adam_m, P) != hipSuccess ||
      hipMalloc(&ctx->adam_v, P) != hipSuccess || hipMalloc(&ctx->grad, P) != hipSuccess ||
      hipMalloc(&ctx->wq, P) != hipSuccess ||
      hipMalloc(&ctx->bias, MLP_NBIAS * sizeof(float)) != hipSuccess ||
      hipMalloc(&ctx->wsw, MLP_SW_SIZE * sizeof(uint16_t)) != hipSuccess ||
      hipMalloc(&ctx->save, 3 * B * 64 * sizeof(float)) != hipSuccess ||
      hipMalloc(&ctx->ybuf, B * MLP_NOUT * sizeof(float)) != hipSuccess ||
      hipMalloc(&ctx->dybuf, B * MLP_NOUT * sizeof(float)) != hipSuccess ||
      hipMalloc(&ctx->delta, B * 200 * sizeof(float)) != hipSuccess ||
      hipMalloc(&ctx->wpart, (size_t)WG_MAXCH * P) != hipSuccess ||
      hipMalloc(&ctx->fitbuf, FIT_DOUBLES * sizeof(double)) != hipSuccess)
    return HRX_ENOMEM;
  if (hipMemset(ctx->adam_m, 0, P) != hipSuccess || hipMemset(ctx->adam_v, 0, P) != hipSuccess)
    return HRX_EHIP;
  ctx->mlp_maxb = max_batch;
  return HRX_OK;
}

int hrx_mlp_set_params(hrx_ctx* ctx, const float* theta, void* hip_stream) {
  if (!ctx || !theta || !ctx->theta) return HRX_EINVAL;
  hipStream_t st = (hipStream_t)hip_stream;
  ctx->last_stream = st;
  const size_t P = MLP_NPARAM * sizeof(float);
  if (hipMemcpyAsync(ctx->theta, theta, P, hipMemcpyDeviceToDevice, st) != hipSuccess ||
      hipMemsetAsync(ctx->adam_m, 0, P, st) != hipSuccess ||
      hipMemsetAsync(ctx->adam_v, 0, P, st) != hipSuccess)
    return HRX_EHIP;
  k_mlp_pack<<<48, 256, 0, st>>>(ctx->theta, ctx->wsw, ctx->bias, ctx->wq);
  ctx->mlp_params = true;
  return check(hipGetLastError());
}

int hrx_mlp_get_params(hrx_ctx* ctx, float* theta_out, void* hip_stream) {
  if (!ctx || !theta_out || !ctx->theta) return HRX_EINVAL;
  hipStream_t st = (hipStream_t)hip_stream;
  ctx->last_stream = st;
  return check(hipMemcpyAsync(theta_out, ctx->theta, MLP_NPARAM * sizeof(float),
                              hipMemcpyDeviceToDevice, st));
}

int hrx_mlp_set_norm(hrx_ctx* ctx, const float* in_mean, const float* in_std,
                     const float* out_mean, const float* out_std, const float* out_lin,
                     double log10rho_min, double log10rho_max, double T_lo, double T_hi,
                     double xiN_min, double xiN_max) {
  if (!ctx || !in_mean || !in_std || !out_mean || !out_std) return HRX_EINVAL;
  if (!(log10rho_min < log10rho_max) || !(T_lo > T_MIN) || !(T_lo < T_hi)) return HRX_EINVAL;
  if (!(xiN_min <= xiN_max)) return HRX_EINVAL;
  MlpNorm nm;
  for (int k = 0; k < MLP_NIN; ++k) {
    if (!(in_std[k] > 0.0f)) return HRX_EINVAL;
    nm.in_mean[k] = in_mean[k];
    nm.in_istd[k] = 1.0f / in_std[k];
  }
  for (int k = 0; k < MLP_NOUT; ++k) {
    if (!(out_std[k] > 0.0f)) return HRX_EINVAL;
    nm.out_mean[k] = out_mean[k];
    nm.out_std[k] = out_std[k];
  }
  for (int o = 0; o < MLP_NOUT; ++o)
    for (int k = 0; k <= MLP_NIN; ++k) nm.out_lin[o][k] = out_lin ? out_lin[o * (MLP_NIN + 1) + k] : 0.0f;
  nm.xiN_min = xiN_min;
  nm.xiN_max = xiN_max;
  nm.log10rho_min = log10rho_min;
  nm.log10rho_max = log10rho_max;
  SpeciesThermo lo, hi;
  species_e_cv(T_lo, lo);
  species_e_cv(T_hi, hi);
  for (int s = 0; s < NS; ++s) {
    nm.e_lo[s] = lo.e[s];
    nm.e_hi[s] = hi.e[s];
  }
  if (!ctx->norm_dev && hipMalloc(&ctx->norm_dev, sizeof(MlpNorm)) != hipSuccess)
    return HRX_ENOMEM;
  // setup call: work still queued on any stream reads the previous statistics first
  int rc = check(hipDeviceSynchronize());
  if (!rc) rc = check(hipMemcpy(ctx->norm_dev, &nm, sizeof(MlpNorm), hipMemcpyHostToDevice));
  if (rc) return rc;
  ctx->mlp_norm = true;
  return HRX_OK;
}

int hrx_mlp_features(hrx_ctx* ctx, int64_t n, const double* rho, const double* e,
                     const double* Y, float* f, void* hip_stream) {
  if (!ctx || n < 0 || (n > 0 && (!rho || !e || !Y || !f))) return HRX_EINVAL;
  if (n == 0) return HRX_OK;
  hipStream_t st = (hipStream_t)hip_stream;
  ctx->last_stream = st;
  k_mlp_features<<<blocks_for(n, 256), 256, 0, st>>>(n, rho, e, Y, f);
  return check(hipGetLastError());
}

int hrx_mlp_dataset(hrx_ctx* ctx, int64_t n, const double* rho, const double* e,
                    const double* Y, double* F, double* T, int32_t* status, void* hip_stream) {
  if (!ctx || n < 0 || (n > 0 && (!rho || !e || !Y || !F || !T))) return HRX_EINVAL;
  if (ctx->cfg.gas != HRX_GAS_AIR5) return HRX_EINVAL;
  if (n == 0) return HRX_OK;
  hipStream_t st = (hipStream_t)hip_stream;
  ctx->last_stream = st;
  k_mlp_dataset<<<blocks_for(n, 128), 128, 0, st>>>(n, ctx->dev.newton_rtol, ctx->dev.newton_max,
                                                    rho, e, Y, F, T, status, ctx->counters);
  return check(hipGetLastError());
}

}  // extern "C"

namespace {
// Eigen-decomposition of a symmetric 8 x 8 matrix by cyclic Jacobi rotations (Golub and
// Van Loan, the symmetric Schur step): A = V diag(lam) V^T, V's columns the eigenvectors.
// A is overwritten.  Returns false when the sweeps do not converge.
bool sym_eigen8(double A[8][8], double V[8][8], double lam[8]) {
  for (int i = 0; i < 8; ++i)
    for (int j = 0; j < 8; ++j) V[i][j] = i == j ? 1.0 : 0.0;
  bool done = false;
  for (int sweep = 0; sweep < 60 && !done; ++sweep) {
    double off = 0.0, dia = 0.0;
    for (int i = 0; i < 8; ++i)
      for (int j = 0; j < 8; ++j) (i == j ? dia : off) += A[i][j] * A[i][j];
    if (!(off <= 1e-28 * dia)) {
      for (int p = 0; p < 7; ++p)
        for (int q = p + 1; q < 8; ++q) {
          if (A[p][q] == 0.0) continue;
          const double tau = (A[q][q] - A[p][p]) / (2.0 * A[p][q]);
          const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
          const double c = 1.0 / sqrt(1.0 + t * t), s = t * c;
          for (int k = 0; k < 8; ++k) {      // A J
            const double akp = A[k][p], akq = A[k][q];
            A[k][p] = c * akp - s * akq;
            A[k][q] = s * akp + c * akq;
          }
          for (int k = 0; k < 8; ++k) {      // J^T A
            const double apk = A[p][k], aqk = A[q][k];
            A[p][k] = c * apk - s * aqk;
            A[q][k] = s * apk + c * aqk;
          }
          for (int k = 0; k < 8; ++k) {      // V J
            const double vkp = V[k][p], vkq = V[k][q];
            V[k][p] = c * vkp - s * vkq;
            V[k][q] = s * vkp + c * vkq;
          }
        }
    } else {
      done = true;
    }
  }
  for (int i = 0; i < 8; ++i) lam[i] = A[i][i];
  return done;
}

// Sums of the wavefront partials of one moments pass (synchronises the stream).
constexpr int FIT_NSV = 2 * MLP_NIN + 64 + 2 * MLP_NOUT, FIT_BLOCKS = 256;
template <int MODE>
int fit_pass(long n, const double* F, const double* Tt, const double* sv_dev, double* part,
             int nblocks, hipStream_t st, std::vector<double>& out) {
  constexpr int K = MODE < 2 ? MLP_NIN : (MODE == 2 ? 36 + 64 : MLP_NOUT);
  k_fit_moments<MODE><<<nblocks, 256, 0, st>>>(n, F, Tt, sv_dev, part);
  int rc = check(hipGetLastError());
  if (rc) return rc;
  const int nw = nblocks * 4;
  std::vector<double> h((size_t)nw * K);
  rc = check(hipMemcpyAsync(h.data(), part, h.size() * sizeof(double), hipMemcpyDeviceToHost, st));
  if (!rc) rc = check(hipStreamSynchronize(st));
  if (rc) return rc;
  out.assign(K, 0.0);
  for (int w = 0; w < nw; ++w)
    for (int k = 0; k < K; ++k) out[k] += h[(size_t)w * K + k];
  return HRX_OK;
}
}  // namespace

extern "C" {

int hrx_mlp_fit(hrx_ctx* ctx, int64_t n, const double* F, const double* T, float* Xs, float* Ys,
                double log10rho_min, double log10rho_max, double T_lo, double T_hi,
                double xiN_min, double xiN_max, double* stats, void* hip_stream) {
  if (!ctx || n < 2 || !F || !T || !Xs || !Ys || !ctx->fitbuf) return HRX_EINVAL;
  hipStream_t st = (hipStream_t)hip_stream;
  ctx->last_stream = st;
  // sv: m [7], 1/s [7], L [8][8], rm [8], 1/rs [8]; then the moments' per-wavefront
  // partials (the context's fit workspace, allocated by hrx_mlp_init)
  constexpr int NSV = FIT_NSV;
  const int nblocks = FIT_BLOCKS;
  double* sv = ctx->fitbuf;
  double* part = ctx->fitbuf + NSV;
  std::vector<double> h(NSV, 0.0), sum;
  auto push = [&]() {
    return check(hipMemcpyAsync(sv, h.data(), NSV * sizeof(double), hipMemcpyHostToDevice, st));
  };
  const double in = 1.0 / (double)n;
  int rc = fit_pass<0>(n, F, T, sv, part, nblocks, st, sum);
  double mean[MLP_NIN], sd[MLP_NIN], L[8][8], rm[MLP_NOUT], rs[MLP_NOUT];
  if (!rc) {
    for (int k = 0; k < MLP_NIN; ++k) h[k] = mean[k] = sum[k] * in;
    rc = push();
  }
  if (!rc) rc = fit_pass<1>(n, F, T, sv, part, nblocks, st, sum);
  if (!rc) {
    for (int k = 0; k < MLP_NIN; ++k) {
      sd[k] = sqrt(sum[k] * in);
      if (!(sd[k] > 0.0)) rc = HRX_EINVAL;
      h[MLP_NIN + k] = 1.0 / sd[k];
    }
    if (!rc) rc = push();
  }
  if (!rc) rc = fit_pass<2>(n, F, T, sv, part, nblocks, st, sum);
  if (!rc) {
    // least squares: the minimum-norm solution of (A^T A) L_o = A^T t_o for every output
    // o.  The five mass fractions sum to one, so A^T A is singular; its directions with an
    // eigenvalue below 1e-9 of the largest are left out (the pseudo-inverse).
    double M[8][8], B[8][8];
    int q = 0;
    for (int p = 0; p < 8; ++p)
      for (int r = p; r < 8; ++r) M[p][r] = M[r][p] = sum[q++];
    for (int o = 0; o < 8; ++o)
      for (int p = 0; p < 8; ++p) B[p][o] = sum[36 + o * 8 + p];
    double V[8][8], lam[8];
    if (!sym_eigen8(M, V, lam)) rc = HRX_EINVAL;
    if (!rc) {
      double lmax = 0.0;
      for (int i = 0; i < 8; ++i) lmax = std::max(lmax, lam[i]);
      if (!(lmax > 0.0)) rc = HRX_EINVAL;
      for (int o = 0; o < 8; ++o)
        for (int p = 0; p < 8; ++p) L[o][p] = 0.0;
      for (int i = 0; i < 8 && !rc; ++i) {
        if (!(lam[i] > 1e-9 * lmax)) continue;
        for (int o = 0; o < 8; ++o) {
          double c = 0.0;
          for (int p = 0; p < 8; ++p) c += V[p][i] * B[p][o];
          c /= lam[i];
          for (int p = 0; p < 8; ++p) L[o][p] += c * V[p][i];
        }
      }
    }
    if (!rc) {
      for (int o = 0; o < 8; ++o)
        for (int p = 0; p < 8; ++p) h[2 * MLP_NIN + o * 8 + p] = L[o][p];
      rc = push();
    }
  }
  if (!rc) rc = fit_pass<3>(n, F, T, sv, part, nblocks, st, sum);
  if (!rc) {
    for (int o = 0; o < MLP_NOUT; ++o) h[2 * MLP_NIN + 64 + o] = rm[o] = sum[o] * in;
    rc = push();
  }
  if (!rc) rc = fit_pass<4>(n, F, T, sv, part, nblocks, st, sum);
  if (!rc) {
    for (int o = 0; o < MLP_NOUT; ++o) {
      rs[o] = sqrt(sum[o] * in);
      if (!(rs[o] > 0.0)) rc = HRX_EINVAL;
      h[2 * MLP_NIN + 72 + o] = 1.0 / rs[o];
    }
    if (!rc) rc = push();
  }
  if (!rc) {
    k_fit_apply<<<blocks_for(n, 256), 256, 0, st>>>(n, F, T, sv, Xs, Ys);
    rc = check(hipGetLastError());
  }
  if (!rc) rc = check(hipStreamSynchronize(st));
  if (rc) return rc;
  // the composition around the network (float, as hrx_mlp_set_norm takes it)
  float fm[MLP_NIN], fs[MLP_NIN], om[MLP_NOUT], os[MLP_NOUT], fl[MLP_NOUT * 8];
  for (int k = 0; k < MLP_NIN; ++k) { fm[k] = (float)mean[k]; fs[k] = (float)sd[k]; }
  for (int o = 0; o < MLP_NOUT; ++o) {
    om[o] = (float)rm[o];
    os[o] = (float)rs[o];
    for (int p = 0; p < 8; ++p) fl[o * 8 + p] = (float)L[o][p];
  }
  if (stats) {
    for (int k = 0; k < MLP_NIN; ++k) { stats[k] = mean[k]; stats[MLP_NIN + k] = sd[k]; }
    for (int o = 0; o < MLP_NOUT; ++o) { stats[14 + o] = rm[o]; stats[22 + o] = rs[o]; }
    for (int o = 0; o < MLP_NOUT; ++o)
      for (int p = 0; p < 8; ++p) stats[30 + o * 8 + p] = L[o][p];
  }
  return hrx_mlp_set_norm(ctx, fm, fs, om, os, fl, log10rho_min, log10rho_max, T_lo, T_hi,
                          xiN_min, xiN_max);
}

int hrx_set_thermo_mode(hrx_ctx* ctx, int mode) {
  if (!ctx) return HRX_EINVAL;
  clear_graphs(ctx);
  if (mode == HRX_THERMO_PLAIN) {
    ctx->thermo_mode = mode;
    return HRX_OK;
  }
  if (mode != HRX_THERMO_SURROGATE || ctx->cfg.gas != HRX_GAS_AIR5) return HRX_EINVAL;
  // the network yields the averaged coefficients of Eq. (19), not the binary ones
  if (ctx->dev.sm) return HRX_EUNSUP;
  if (!ctx->mlp_params || !ctx->mlp_norm) return HRX_EINVAL;
  const int rc = ensure_ys(ctx, std::max<int64_t>(ctx->dev.N, THERMO_CHUNK));
  if (rc) return rc;
  ctx->thermo_mode = mode;
  return HRX_OK;
}

int hrx_mlp_forward(hrx_ctx* ctx, int64_t n, const float* X, float* Y, void* hip_stream) {
  if (!ctx || n < 0 || (n > 0 && (!X || !Y)) || !ctx->mlp_params) return HRX_EINVAL;
  if (n == 0) return HRX_OK;
  hipStream_t st = (hipStream_t)hip_stream;
  ctx->last_stream = st;
  const unsigned nb = (unsigned)std::min<int64_t>((n + 255) / 256, 2048);
  k_mlp_fwd<<<nb, 256, 0, st>>>(n, X, nullptr, Y, nullptr, ctx->wsw, ctx->bias);
  return check(hipGetLastError());
}

static void launch_wgrad(hrx_ctx* ctx, int64_t n, const float* X, const int32_t* idx,
                         float* grad, hipStream_t st) {
  const int64_t nch = std::min<int64_t>(WG_MAXCH, (n + 255) / 256);
  const int64_t cb = (n + nch - 1) / nch;
  k_mlp_wgrad<<<dim3((unsigned)nch, 4), 256, 0, st>>>(n, cb, X, idx, ctx->save, ctx->delta,
                                                       ctx->wpart);
  k_mlp_wgrad_sum<<<blocks_for(MLP_NPARAM, 256), 256, 0, st>>>((int)nch, ctx->wpart, grad);
}

static int mlp_backward_impl(hrx_ctx* ctx, int64_t n, const int32_t* idx, const float* X,
                             const float* dY, float* grad, hipStream_t st) {
  const unsigned nb = (unsigned)std::min<int64_t>((n + 255) / 256, 2048);
  k_mlp_fwd<<<nb, 256, 0, st>>>(n, X, idx, ctx->ybuf, ctx->save, ctx->wsw, ctx->bias);
  k_mlp_bwd_delta<<<blocks_for(n, 128), 128, 0, st>>>(n, dY, ctx->save, ctx->wq, ctx->delta);
  launch_wgrad(ctx, n, X, idx, grad, st);
  return check(hipGetLastError());
}

int hrx_mlp_backward(hrx_ctx* ctx, int64_t n, const float* X, const float* dLdY, float* grad,
                     void* hip_stream) {
  if (!ctx || !ctx->mlp_params || n < 1 || n > ctx->mlp_maxb || !X || !dLdY || !grad)
    return HRX_EINVAL;
  hipStream_t st = (hipStream_t)hip_stream;
  ctx->last_stream = st;
  return mlp_backward_impl(ctx, n, nullptr, X, dLdY, grad, st);
}

int hrx_adam_step(hrx_ctx* ctx, const float* grad, float lr, int t, void* hip_stream) {
  if (!ctx || !ctx->mlp_params || !grad || t < 1 || !(lr >= 0.0f)) return HRX_EINVAL;
  hipStream_t st = (hipStream_t)hip_stream;
  ctx->last_stream = st;
  const float bc1 = (float)(1.0 - pow(0.9, t)), bc2 = (float)(1.0 - pow(0.999, t));
  k_adam<<<blocks_for(MLP_NPARAM, 256), 256, 0, st>>>(ctx->theta, ctx->adam_m, ctx->adam_v, grad,
                                                      lr, bc1, bc2);
  k_mlp_pack<<<48, 256, 0, st>>>(ctx->theta, ctx->wsw, ctx->bias, ctx->wq);
  return check(hipGetLastError());
}

int hrx_mlp_train_step(hrx_ctx* ctx, int64_t n, const int32_t* idx, const float* X,
                       const float* Yt, float lr, int t, float* loss, void* hip_stream) {
  if (!ctx || !ctx->mlp_params || n < 1 || n > ctx->mlp_maxb || !X || !Yt || t < 1)
    return HRX_EINVAL;
  hipStream_t st = (hipStream_t)hip_stream;
  ctx->last_stream = st;
  const unsigned nb = (unsigned)std::min<int64_t>((n + 255) / 256, 2048);
  k_mlp_fwd<<<nb, 256, 0, st>>>(n, X, idx, ctx->ybuf, ctx->save, ctx->wsw, ctx->bias);
  k_mlp_mse<<<(unsigned)std::min<int64_t>((n * MLP_NOUT + 255) / 256, 1024), 256, 0, st>>>(
      n, ctx->ybuf, Yt, idx, ctx->dybuf, loss);
  k_mlp_bwd_delta<<<blocks_for(n, 128), 128, 0, st>>>(n, ctx->dybuf, ctx->save, ctx->wq,
                                                      ctx->delta);
  launch_wgrad(ctx, n, X, idx, ctx->grad, st);
  int rc = check(hipGetLastError());
  if (rc) return rc;
  return hrx_adam_step(ctx, ctx->grad, lr, t, hip_stream);
}

}  // extern "C"
