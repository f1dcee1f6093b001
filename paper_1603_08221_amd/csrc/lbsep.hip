// lbsep: fused sweep kernel and host implementation of include/lbsep.h.
//
// One time step = one launch of k_sweep<T, /*PULL=*/true, /*EVAL=*/false>:
// every thread owns one node (x, j) and
//   1. pulls the 18 post-collision populations of the previous step from its
//      neighbours (Eq. (MRT), pull form of the streaming),
//   2. replaces the wall-crossing pulls by diffuse-bounce-back (Eqs. (bot),
//      (bot2)) from its own post-collision populations,
//   3. on the inlet/outlet columns, rebuilds the node from the first and second
//      inner layers scaled by the column density correction (Eqs. (rho1), (rho2)),
//   4. computes moments (Eq. (rhou)), relaxation times (Eqs. (taos), (EQFrsp),
//      (taoq)) and collides both species (Eq. (MR)),
//   5. writes the 18 new post-collision populations, and
//   6. adds its species number density and x-momentum to FP64 column sums,
//      reduced to C_l(x), CL and C~_l (Eqs. (C), (CL), (Clline)) by the last
//      block to finish (no second launch, deterministic summation order).
//
// Layout in HBM (structure of arrays): population (s, i) of node (x, j) of a
// state buffer is at element ((s * 9 + i) * ny + j) * pitch + x, pitch =
// nx rounded up to 64, so a wavefront reads 64 consecutive x of one row.
// Two state buffers alternate; the one written last holds the post-collision
// state f'(t), the other the previous post-collision state f'(t-1) (or, right
// after init / set_state, the pre-collision state f(t)).
//
// Work decomposition: a block is 4 wavefronts = 64 columns x (4 * rpt) rows.
// Blocks 0 and 1 own the inlet and outlet columns (they need whole-column sums
// of the inner layers before they can rebuild the boundary nodes); blocks
// 2..7 are idle; tiles follow, numbered so that each XCD (block id mod 8)
// takes a contiguous run of tiles, vertically adjacent tiles first, which
// keeps the halo rows of a tile in the same XCD's L2.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>

#include "lbsep.h"
#include "lbsep_device.h"

namespace lbsep {
namespace {

constexpr int kTX = 64;         // columns per block (one wavefront across x)
constexpr int kTY = 4;          // wavefronts per block
constexpr int kThreads = kTX * kTY;
constexpr int kLeadBlocks = 8;  // blocks 0..7: inlet, outlet, idle

struct KParams {
  RelaxConsts rc;
  int nx, ny, pitch;
  int nxt, nrt, rpt;  // column strips, row tiles, rows per thread
  int tiles, chunk;   // nxt * nrt, ceil(tiles / 8)
  long long plane;    // ny * pitch
  unsigned flags;
  double r;           // DBB coefficient
  double rho_bc[2][2];  // [inlet/outlet][species] densities of Eq. (rho2)
  double cl_in;
};

struct KBufs {
  double* partials;    // [4][nrt][pitch] per row-tile column sums
  double* endsum;      // [2][4] inlet / outlet column sums
  double* colsum;      // [4][pitch] column sums of the last recorded state
  double* strip;       // [nxt][4] (min C_l, argmin, sum (C_l - C_in), bad)
  double* hist;        // [hist_cap][4] (t, CL, C~_l, x_min)
  unsigned* counters;  // [nxt + 1] arrival counters (strips, then global)
  unsigned* status;    // [1] bit 0: non-finite or non-positive column density seen
  long long hist_cap;
};

__device__ __forceinline__ long long pidx(const KParams& kp, int s, int i, int j, int x) {
  return (long long)(s * 9 + i) * kp.plane + (long long)j * kp.pitch + x;
}

// Pre-collision populations of node (x, j) at the new time level.
// PULL: streamed from the post-collision state in src, with DBB on wall rows.
// !PULL: read in place (src already holds a pre-collision state).
template <typename T, bool PULL>
__device__ __forceinline__ void gather(const KParams& kp, const T* __restrict__ src, int x, int j, T fa[9],
                                       T fb[9]) {
  if (!PULL) {
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      fa[i] = src[pidx(kp, 0, i, j, x)];
      fb[i] = src[pidx(kp, 1, i, j, x)];
    }
    return;
  }
  int xm = x - 1, xp = x + 1, jm = j - 1, jp = j + 1;
  if (kp.flags & LBSEP_PERIODIC_X) {
    if (xm < 0) xm += kp.nx;
    if (xp >= kp.nx) xp -= kp.nx;
  }
  bool bot = false, top = false;
  if (kp.flags & LBSEP_PERIODIC_Y) {
    if (jm < 0) jm += kp.ny;
    if (jp >= kp.ny) jp -= kp.ny;
  } else {
    bot = (j == 0);
    top = (j == kp.ny - 1);
    // keep the (discarded) wall-crossing loads in range
    if (bot) jm = j;
    if (top) jp = j;
  }
  // source of direction i is (x - c_ix, j - c_iy)
  const int sx[9] = {x, xm, x, xp, x, xm, xp, xp, xm};
  const int sy[9] = {j, j, jm, j, jp, jm, jm, jp, jp};
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    fa[i] = src[pidx(kp, 0, i, sy[i], sx[i])];
    fb[i] = src[pidx(kp, 1, i, sy[i], sx[i])];
  }
  if (bot || top) {
    // Eqs. (bot)/(bot2): the populations that would come from outside the
    // channel are r f^eq(rho_w, u_w = 0) + (1 - r) f'_opposite at the same node;
    // rho_w makes the returned mass equal the leaving mass F, which puts the
    // shares 4/6, 1/6, 1/6 of F on the axis and the two diagonal directions.
    const T r = T(kp.r);
    const T q = T(1) - r;
    const int o0 = bot ? 4 : 2, o1 = bot ? 7 : 5, o2 = bot ? 8 : 6;  // leaving
    const int u0 = bot ? 2 : 4, u1 = bot ? 5 : 7, u2 = bot ? 6 : 8;  // returning
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      T* f = s ? fb : fa;
      const T l0 = src[pidx(kp, s, o0, j, x)];
      const T l1 = src[pidx(kp, s, o1, j, x)];
      const T l2 = src[pidx(kp, s, o2, j, x)];
      const T F = l0 + l1 + l2;
      f[u0] = r * (T(2.0 / 3.0) * F) + q * l0;
      f[u1] = r * (F * T(1.0 / 6.0)) + q * l1;
      f[u2] = r * (F * T(1.0 / 6.0)) + q * l2;
    }
  }
}

template <typename T>
__device__ __forceinline__ T sum9(const T f[9]) {
  return ((f[0] + f[1]) + (f[2] + f[3])) + ((f[4] + f[5]) + (f[6] + f[7])) + f[8];
}

// Moments, relaxation times and (STEP) collision + store or (EVAL) output of
// one node. acc receives (n_a, n_b, rho_a u_ax, rho_b u_bx) in double.
template <typename T, bool EVAL>
__device__ __forceinline__ void process_node(const KParams& kp, int x, int j, T fa[9], T fb[9],
                                             T* __restrict__ dst, double* __restrict__ mom,
                                             T* __restrict__ fout, double acc[4]) {
  const T rho_a = sum9(fa);
  const T rho_b = sum9(fb);
  const T jxa = (fa[1] - fa[3]) + (fa[5] - fa[6]) + (fa[8] - fa[7]);
  const T jya = (fa[2] - fa[4]) + (fa[5] + fa[6]) - (fa[7] + fa[8]);
  const T jxb = (fb[1] - fb[3]) + (fb[5] - fb[6]) + (fb[8] - fb[7]);
  const T jyb = (fb[2] - fb[4]) + (fb[5] + fb[6]) - (fb[7] + fb[8]);
  const T rho = rho_a + rho_b;
  const T inv_rho = T(1) / rho;
  const T ux = (jxa + jxb) * inv_rho;
  const T uy = (jya + jyb) * inv_rho;
  T ts, td, tq;
  relaxation_times<T>(kp.rc, j, rho_a, rho_b, ts, td, tq);
  // species momentum of Eq. (rhou): rho_s u_s = (1 - 1/(2 tau_d)) j_s + rho_s u / (2 tau_d)
  const T h2 = T(0.5) / td;
  const T g = T(1) - h2;
  const T pxa = g * jxa + rho_a * ux * h2;
  const T pxb = g * jxb + rho_b * ux * h2;
  if (EVAL) {
    const long long n = (long long)kp.nx * kp.ny;
    const long long o = (long long)j * kp.nx + x;
    if (mom) {
      const T pya = g * jya + rho_a * uy * h2;
      const T pyb = g * jyb + rho_b * uy * h2;
      mom[o] = double(rho_a);
      mom[n + o] = double(rho_b);
      mom[2 * n + o] = double(pxa / rho_a);
      mom[3 * n + o] = double(pya / rho_a);
      mom[4 * n + o] = double(pxb / rho_b);
      mom[5 * n + o] = double(pyb / rho_b);
    }
    if (fout) {
#pragma unroll
      for (int i = 0; i < 9; ++i) {
        fout[i * n + o] = fa[i];
        fout[(9 + i) * n + o] = fb[i];
      }
    }
    return;
  }
  acc[0] += double(rho_a) * kp.rc.inv_m[0];
  acc[1] += double(rho_b) * kp.rc.inv_m[1];
  acc[2] += double(pxa);
  acc[3] += double(pxb);
  T we, weps;
  if (kp.rc.bgk) {
    we = weps = T(1) / ts;
  } else {
    we = T(1.0 / 1.1);     // tau_e = 1.1 (Sec. 3.3)
    weps = T(1.0 / 1.2);   // tau_eps = 1.2
  }
  const T wd = T(1) / td, wq = T(1) / tq, ws = T(1) / ts;
  collide_species<T>(fa, rho_a, ux, uy, T(kp.rc.s[0]), we, weps, wd, wq, ws);
  collide_species<T>(fb, rho_b, ux, uy, T(kp.rc.s[1]), we, weps, wd, wq, ws);
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    dst[pidx(kp, 0, i, j, x)] = fa[i];
    dst[pidx(kp, 1, i, j, x)] = fb[i];
  }
}

// Last-arriver detection for the block-level reduction. Every thread fences
// its own stores before the block's single arrival; the last block fences
// again before it reads what the others wrote.
__device__ __forceinline__ bool arrive_last(unsigned* counter, unsigned expected) {
  __shared__ int last;
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned prev = atomicAdd(counter, 1u);
    last = (prev == expected - 1u);
  }
  __syncthreads();
  const bool is_last = last != 0;
  if (is_last) __threadfence();
  return is_last;
}

// Reduction of one column strip (64 columns) after all its row tiles (and the
// inlet/outlet block that owns one of its columns) have stored their sums,
// then, for the last strip, of all strips to CL and C~_l for level t.
__device__ void finish_strip(const KParams& kp, const KBufs& kb, int bx, long long t,
                             double (*red)[kTY][kTX]) {
  const int tx = threadIdx.x & (kTX - 1);
  const int q = threadIdx.x / kTX;  // which sum
  const int x = bx * kTX + tx;
  const bool px = kp.flags & LBSEP_PERIODIC_X;
  double v = 0.0;
  if (x < kp.nx) {
    if (!px && x == 0) {
      v = kb.endsum[0 * 4 + q];
    } else if (!px && x == kp.nx - 1) {
      v = kb.endsum[1 * 4 + q];
    } else {
      const double* p = kb.partials + (long long)q * kp.nrt * kp.pitch + x;
      for (int by = 0; by < kp.nrt; ++by) v += p[(long long)by * kp.pitch];
    }
    kb.colsum[(long long)q * kp.pitch + x] = v;
  }
  red[q][0][tx] = v;
  __syncthreads();
  if (q == 0) {
    double cl = 1e300, dev = 0.0, arg = 1e300;
    double bad = 0.0;
    if (x < kp.nx) {
      const double na = red[0][0][tx], nb = red[1][0][tx];
      cl = na / (na + nb);
      dev = cl - kp.cl_in;
      arg = double(x);
      const bool ok = (na > 0.0) && (nb > 0.0) && isfinite(na + nb) && isfinite(red[2][0][tx]) &&
                      isfinite(red[3][0][tx]);
      bad = ok ? 0.0 : 1.0;
      if (!ok) cl = -1e300;  // keep a bad column visible in the minimum
    }
    // wavefront tree reductions: min (ties -> smaller x), sum, max
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
      const double ocl = __shfl_xor(cl, off);
      const double oarg = __shfl_xor(arg, off);
      const double odev = __shfl_xor(dev, off);
      const double obad = __shfl_xor(bad, off);
      if (ocl < cl || (ocl == cl && oarg < arg)) {
        cl = ocl;
        arg = oarg;
      }
      dev += odev;
      bad = fmax(bad, obad);
    }
    if (tx == 0) {
      double* s = kb.strip + (long long)bx * 4;
      s[0] = cl;
      s[1] = arg;
      s[2] = dev;
      s[3] = bad;
      kb.counters[bx] = 0u;  // all arrivals for this strip are in
    }
  }
  if (!arrive_last(kb.counters + kp.nxt, (unsigned)kp.nxt)) return;
  if (threadIdx.x < kTX) {
    const int lane = threadIdx.x;
    double cl = 1e300, arg = 1e300, dev = 0.0, bad = 0.0;
    for (int k = lane; k < kp.nxt; k += kTX) {
      const double* s = kb.strip + (long long)k * 4;
      if (s[0] < cl || (s[0] == cl && s[1] < arg)) {
        cl = s[0];
        arg = s[1];
      }
      dev += s[2];
      bad = fmax(bad, s[3]);
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
      const double ocl = __shfl_xor(cl, off);
      const double oarg = __shfl_xor(arg, off);
      const double odev = __shfl_xor(dev, off);
      const double obad = __shfl_xor(bad, off);
      if (ocl < cl || (ocl == cl && oarg < arg)) {
        cl = ocl;
        arg = oarg;
      }
      dev += odev;
      bad = fmax(bad, obad);
    }
    if (lane == 0) {
      double* h = kb.hist + (t % kb.hist_cap) * 4;
      h[0] = double(t);
      h[1] = (kp.cl_in - cl) / kp.cl_in;                 // Eq. (CL)
      h[2] = dev / (double(kp.nx) * kp.cl_in);           // Eq. (Clline)
      h[3] = arg;
      if (bad != 0.0) atomicOr(kb.status, 1u);
      kb.counters[kp.nxt] = 0u;
    }
  }
}

// Block-wide sum of nv <= 4 doubles per thread (fixed order); the result for
// quantity k is left in red[k][0][0]. Every thread reaches every barrier.
__device__ void block_sum(double (*red)[kTY][kTX], const double* v, int nv) {
  const int tx = threadIdx.x & (kTX - 1);
  const int w = threadIdx.x / kTX;
  for (int k = 0; k < nv; ++k) red[k][w][tx] = v[k];
  __syncthreads();
  const int k = w;  // wavefront w sums quantity k = w (wave-uniform)
  double s = 0.0;
  if (k < nv) {
    s = ((red[k][0][tx] + red[k][1][tx]) + red[k][2][tx]) + red[k][3][tx];
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off);
  }
  __syncthreads();
  if (k < nv && tx == 0) red[k][0][0] = s;
  __syncthreads();
}

template <typename T, bool PULL, bool EVAL>
__global__ __launch_bounds__(kThreads) void k_sweep(KParams kp, KBufs kb, const T* __restrict__ src,
                                                    T* __restrict__ dst, double* __restrict__ mom,
                                                    T* __restrict__ fout, long long t) {
  __shared__ double red[4][kTY][kTX];
  const int b = blockIdx.x;
  const bool px = kp.flags & LBSEP_PERIODIC_X;
  if (b < kLeadBlocks) {
    // ---- inlet (b = 0) / outlet (b = 1) column ---------------------------
    if (px || b >= 2) return;
    const int e = b;
    const int col = e ? kp.nx - 1 : 0;
    const int l1 = e ? kp.nx - 2 : 1;
    const int l2 = e ? kp.nx - 3 : 2;
    T kap[2] = {T(1), T(1)};
    if (PULL) {
      // Eq. (rho1): rho'(col, j) = 2 rho(l1, j) - rho(l2, j); Eq. (rho2): kappa
      double sums[2] = {0.0, 0.0};
      for (int j = threadIdx.x; j < kp.ny; j += kThreads) {
        T fa[9], fb[9], ga[9], gb[9];
        gather<T, true>(kp, src, l1, j, fa, fb);
        gather<T, true>(kp, src, l2, j, ga, gb);
        sums[0] += double(T(2) * sum9(fa) - sum9(ga));
        sums[1] += double(T(2) * sum9(fb) - sum9(gb));
      }
      block_sum(red, sums, 2);
      kap[0] = T(double(kp.ny) * kp.rho_bc[e][0] / red[0][0][0]);
      kap[1] = T(double(kp.ny) * kp.rho_bc[e][1] / red[1][0][0]);
      __syncthreads();
    }
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int j = threadIdx.x; j < kp.ny; j += kThreads) {
      T fa[9], fb[9];
      if (PULL) {
        T ga[9], gb[9];
        gather<T, true>(kp, src, l1, j, fa, fb);
        gather<T, true>(kp, src, l2, j, ga, gb);
#pragma unroll
        for (int i = 0; i < 9; ++i) {
          fa[i] = kap[0] * (T(2) * fa[i] - ga[i]);
          fb[i] = kap[1] * (T(2) * fb[i] - gb[i]);
        }
      } else {
        gather<T, false>(kp, src, col, j, fa, fb);
      }
      process_node<T, EVAL>(kp, col, j, fa, fb, dst, mom, fout, acc);
    }
    if (EVAL) return;
    block_sum(red, acc, 4);
    if (threadIdx.x < 4) kb.endsum[e * 4 + threadIdx.x] = red[threadIdx.x][0][0];
    __syncthreads();
    const int bx = e ? kp.nxt - 1 : 0;
    const unsigned expected = (unsigned)kp.nrt + 1u + ((kp.nxt == 1) ? 1u : 0u);
    if (arrive_last(kb.counters + bx, expected)) finish_strip(kp, kb, bx, t, red);
    return;
  }
  // ---- interior tile ---------------------------------------------------------
  const int xcd = b & 7;
  const int k = (b >> 3) - 1;
  const int lin = xcd * kp.chunk + k;
  if (lin >= kp.tiles) return;
  const int bx = lin / kp.nrt;
  const int by = lin - bx * kp.nrt;
  const int tx = threadIdx.x & (kTX - 1);
  const int ty = threadIdx.x / kTX;
  const int x = bx * kTX + tx;
  const bool xin = (x < kp.nx) && (px || (x > 0 && x < kp.nx - 1));
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int r = 0; r < kp.rpt; ++r) {
    const int j = by * (kTY * kp.rpt) + r * kTY + ty;
    if (xin && j < kp.ny) {
      T fa[9], fb[9];
      gather<T, PULL>(kp, src, x, j, fa, fb);
      process_node<T, EVAL>(kp, x, j, fa, fb, dst, mom, fout, acc);
    }
  }
  if (EVAL) return;
  // per-column sums of this row tile (4 wavefronts -> 1), quantity q = ty
#pragma unroll
  for (int q = 0; q < 4; ++q) red[q][ty][tx] = acc[q];
  __syncthreads();
  if (x < kp.nx) {
    const double s = ((red[ty][0][tx] + red[ty][1][tx]) + red[ty][2][tx]) + red[ty][3][tx];
    kb.partials[((long long)ty * kp.nrt + by) * kp.pitch + x] = s;
  }
  const unsigned expected =
      (unsigned)kp.nrt + ((!px && bx == 0) ? 1u : 0u) + ((!px && bx == kp.nxt - 1) ? 1u : 0u);
  if (arrive_last(kb.counters + bx, expected)) finish_strip(kp, kb, bx, t, red);
}

// Initial state: f = f^eq(rho_s(x), u = 0) (Eq. (feq) at rest), pressure and
// C_l linear in x from (P_in, C_in) to (P_out, C_out).
template <typename T>
__global__ __launch_bounds__(kThreads) void k_init(KParams kp, T* __restrict__ f, double p_in, double p_out,
                                                   double c_in, double c_out) {
  const long long n = (long long)kp.ny * kp.pitch;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (long long)gridDim.x * blockDim.x) {
    const int j = int(e / kp.pitch);
    const int x = int(e - (long long)j * kp.pitch);
    if (x >= kp.nx) continue;
    const double frac = kp.nx > 1 ? double(x) / double(kp.nx - 1) : 0.0;
    const double p = p_in + (p_out - p_in) * frac;
    const double c = c_in + (c_out - c_in) * frac;
    const double rho[2] = {c * p / (kp.rc.s[0] * (1.0 / 3.0)), (1.0 - c) * p / (kp.rc.s[1] * (1.0 / 3.0))};
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const double sv = kp.rc.s[s];
      const double a0 = (9.0 - 5.0 * sv) / 4.0;
      f[pidx(kp, s, 0, j, x)] = T(4.0 / 9.0 * rho[s] * a0);
#pragma unroll
      for (int i = 1; i < 5; ++i) f[pidx(kp, s, i, j, x)] = T(1.0 / 9.0 * rho[s] * sv);
#pragma unroll
      for (int i = 5; i < 9; ++i) f[pidx(kp, s, i, j, x)] = T(1.0 / 36.0 * rho[s] * sv);
    }
  }
}

__global__ void k_zero_u32(unsigned* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

// Dense [2*9*ny][nx] <-> pitched state copy.
template <typename T>
__global__ void k_copy_in(KParams kp, const T* __restrict__ dense, T* __restrict__ f) {
  const long long n = 18LL * kp.ny * kp.nx;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (long long)gridDim.x * blockDim.x) {
    const long long row = e / kp.nx;
    const int x = int(e - row * kp.nx);
    f[row * kp.pitch + x] = dense[e];
  }
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

struct Layout {
  int pitch, nxt, nrt, rpt, tiles, chunk;
  size_t elem, state_buf, f0, f1, partials, endsum, colsum, strip, hist, counters, mom, total;
};

bool validate(const lbsep_params* p, std::string& why) {
  if (!p) return why = "params is NULL", false;
  const bool px = p->flags & LBSEP_PERIODIC_X;
  const bool py = p->flags & LBSEP_PERIODIC_Y;
  if (p->flags & ~0xFu) return why = "unknown flag bits", false;
  if (p->nx < (px ? 1 : 6)) return why = "nx must be >= 6 (>= 1 with LBSEP_PERIODIC_X)", false;
  if (p->ny < 2) return why = "ny must be >= 2", false;
  if ((long long)p->nx * p->ny > (1LL << 31)) return why = "nx * ny too large", false;
  if (!(p->m_a > 0) || !(p->m_b >= p->m_a) || !std::isfinite(p->m_b))
    return why = "need 0 < m_a <= m_b (species a is the light one)", false;
  if (!(p->cl_in > 0 && p->cl_in < 1) || !(p->cl_out > 0 && p->cl_out < 1))
    return why = "cl_in and cl_out must be in (0, 1)", false;
  if (!(p->theta > 0) || !std::isfinite(p->theta)) return why = "theta must be > 0", false;
  if (!(p->kn_out > 0) || !std::isfinite(p->kn_out)) return why = "kn_out must be > 0", false;
  if (!(p->dbb_r >= 0 && p->dbb_r < 2)) return why = "dbb_r must be in [0, 2)", false;
  if (!(p->accom > 0 && p->accom <= 1)) return why = "accom must be in (0, 1]", false;
  if ((p->flags & LBSEP_BGK_TEST) && !(p->tau_bgk > 0.5 && std::isfinite(p->tau_bgk)))
    return why = "tau_bgk must be > 0.5 with LBSEP_BGK_TEST", false;
  if (py && !(p->flags & LBSEP_MFP_OFF)) return why = "LBSEP_PERIODIC_Y requires LBSEP_MFP_OFF", false;
  if (p->dtype != LBSEP_F64 && p->dtype != LBSEP_F32) return why = "dtype must be LBSEP_F64 or LBSEP_F32", false;
  if (p->hist_cap < 1) return why = "hist_cap must be >= 1", false;
  return true;
}

Layout make_layout(const lbsep_params* p) {
  Layout L{};
  L.elem = p->dtype == LBSEP_F64 ? sizeof(double) : sizeof(float);
  L.pitch = (int)align_up((size_t)p->nx, kTX);
  L.nxt = (p->nx + kTX - 1) / kTX;
  // rows per thread: the largest of 4, 2, 1 that still gives >= 1024 tiles
  L.rpt = 1;
  for (int r : {4, 2}) {
    const int nrt = (p->ny + kTY * r - 1) / (kTY * r);
    if ((long long)L.nxt * nrt >= 1024) {
      L.rpt = r;
      break;
    }
  }
  L.nrt = (p->ny + kTY * L.rpt - 1) / (kTY * L.rpt);
  L.tiles = L.nxt * L.nrt;
  L.chunk = (L.tiles + 7) / 8;
  L.state_buf = align_up(18ull * p->ny * L.pitch * L.elem, 256);
  size_t off = 0;
  L.f0 = off; off += L.state_buf;
  L.f1 = off; off += L.state_buf;
  L.partials = off; off += align_up(4ull * L.nrt * L.pitch * sizeof(double), 256);
  L.endsum = off; off += 256;
  L.colsum = off; off += align_up(4ull * L.pitch * sizeof(double), 256);
  L.strip = off; off += align_up(4ull * L.nxt * sizeof(double), 256);
  L.hist = off; off += align_up(4ull * p->hist_cap * sizeof(double), 256);
  L.counters = off; off += align_up((L.nxt + 2ull) * sizeof(unsigned), 256);
  L.mom = off; off += align_up(6ull * p->ny * p->nx * sizeof(double), 256);
  L.total = off;
  return L;
}

}  // namespace
}  // namespace lbsep

using namespace lbsep;

struct lbsep_channel {
  lbsep_params p;
  Layout L;
  KParams kp;
  KBufs kb;
  hipStream_t stream;
  char* ws;
  void* f[2];
  double* mom;
  int cur;        // buffer holding f'(t)
  bool prev_pre;  // the other buffer holds the pre-collision f(t) (after init / set_state)
  int64_t t;
  int64_t t_first;  // first level with a history record
};

namespace {

int check_hip(hipError_t e, const char* what) {
  if (e != hipSuccess) return fail(LBSEP_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
  return LBSEP_OK;
}

template <typename T, bool PULL, bool EVAL>
void launch_sweep(lbsep_channel* h, const void* src, void* dst, double* mom, void* fout, long long t) {
  const int grid = kLeadBlocks + 8 * h->L.chunk;
  hipLaunchKernelGGL((k_sweep<T, PULL, EVAL>), dim3(grid), dim3(kThreads), 0, h->stream, h->kp, h->kb,
                     static_cast<const T*>(src), static_cast<T*>(dst), mom, static_cast<T*>(fout), t);
}

template <bool PULL, bool EVAL>
void sweep_any(lbsep_channel* h, const void* src, void* dst, double* mom, void* fout, long long t) {
  if (h->p.dtype == LBSEP_F64)
    launch_sweep<double, PULL, EVAL>(h, src, dst, mom, fout, t);
  else
    launch_sweep<float, PULL, EVAL>(h, src, dst, mom, fout, t);
}

// Collide the pre-collision state held in f[0] into f[1] at level t.
int collide_loaded(lbsep_channel* h, int64_t t) {
  sweep_any<false, false>(h, h->f[0], h->f[1], nullptr, nullptr, t);
  h->cur = 1;
  h->prev_pre = true;
  h->t = t;
  h->t_first = t;
  return check_hip(hipGetLastError(), "collide launch");
}

// EVAL sweep of the current state into mom and/or fout.
int eval_state(lbsep_channel* h, double* mom, void* fout) {
  const void* prev = h->f[1 - h->cur];
  if (h->prev_pre)
    sweep_any<false, true>(h, prev, nullptr, mom, fout, h->t);
  else
    sweep_any<true, true>(h, prev, nullptr, mom, fout, h->t);
  return check_hip(hipGetLastError(), "eval launch");
}

}  // namespace

extern "C" {

const char* lbsep_last_error(void) { return g_err.c_str(); }

size_t lbsep_workspace_bytes(const lbsep_params* p) {
  std::string why;
  if (!validate(p, why)) {
    fail(LBSEP_EINVAL, why);
    return 0;
  }
  return make_layout(p).total;
}

size_t lbsep_state_bytes(const lbsep_params* p) {
  std::string why;
  if (!validate(p, why)) {
    fail(LBSEP_EINVAL, why);
    return 0;
  }
  return 18ull * p->ny * p->nx * (p->dtype == LBSEP_F64 ? sizeof(double) : sizeof(float));
}

double lbsep_dbb_r_from_cm(double c_m, double m_a, double m_b, double cl) {
  if (!(c_m >= 0) || !(m_a > 0) || !(m_b > 0) || !(cl >= 0 && cl <= 1)) return NAN;
  const double m_min = m_a < m_b ? m_a : m_b;
  const double m_x = cl * m_a + (1.0 - cl) * m_b;
  const double kbt = m_min / 3.0;
  return 2.0 - 2.0 / (1.0 + (c_m / 3.0) * std::sqrt(M_PI * m_x / (2.0 * kbt)));
}

int lbsep_init(const lbsep_params* p, void* dev_ws, size_t ws_bytes, void* hip_stream, lbsep_channel** out) {
  if (!out) return fail(LBSEP_EINVAL, "out is NULL");
  *out = nullptr;
  std::string why;
  if (!validate(p, why)) return fail(LBSEP_EINVAL, why);
  if (!dev_ws || (reinterpret_cast<uintptr_t>(dev_ws) & 255u))
    return fail(LBSEP_EINVAL, "dev_ws must be a non-NULL 256-byte aligned device pointer");
  const Layout L = make_layout(p);
  if (ws_bytes < L.total)
    return fail(LBSEP_ESIZE, "workspace too small: need " + std::to_string(L.total) + " bytes");
  lbsep_channel* h = new (std::nothrow) lbsep_channel();
  if (!h) return fail(LBSEP_EDEVICE, "out of host memory");
  h->p = *p;
  h->L = L;
  h->stream = static_cast<hipStream_t>(hip_stream);
  h->ws = static_cast<char*>(dev_ws);
  h->f[0] = h->ws + L.f0;
  h->f[1] = h->ws + L.f1;
  h->mom = reinterpret_cast<double*>(h->ws + L.mom);

  KParams& kp = h->kp;
  const double m_min = p->m_a;  // validated: m_a <= m_b
  const double cs2 = 1.0 / 3.0, p_out = cs2, p_in = p->theta * cs2;
  kp.nx = p->nx;
  kp.ny = p->ny;
  kp.pitch = L.pitch;
  kp.nxt = L.nxt;
  kp.nrt = L.nrt;
  kp.rpt = L.rpt;
  kp.tiles = L.tiles;
  kp.chunk = L.chunk;
  kp.plane = (long long)p->ny * L.pitch;
  kp.flags = p->flags;
  kp.r = p->dbb_r;
  kp.cl_in = p->cl_in;
  RelaxConsts& rc = kp.rc;
  rc.inv_m[0] = 1.0 / p->m_a;
  rc.inv_m[1] = 1.0 / p->m_b;
  rc.s[0] = m_min / p->m_a;
  rc.s[1] = m_min / p->m_b;
  rc.lam_p = p->kn_out * double(p->ny) * p_out;
  rc.kpref = std::sqrt(6.0 * m_min / M_PI);
  rc.dpref = 1.5 * std::sqrt(3.0 * (p->m_a + p->m_b) * p->m_a * p->m_b / m_min);
  const double a1 = (2.0 - p->accom) / p->accom * (1.0 - 0.1817 * p->accom);  // Eq. (A12)
  const double a2 = 1.0 / M_PI + 0.5 * a1 * a1;
  const double vs = std::sqrt(M_PI / 6.0);
  rc.tq_a = 24.0 * vs * vs * a2;
  rc.tq_b = 30.0 * vs * a1;
  rc.height = double(p->ny);
  rc.tau_bgk = p->tau_bgk;
  rc.mfp_off = (p->flags & LBSEP_MFP_OFF) ? 1 : 0;
  rc.bgk = (p->flags & LBSEP_BGK_TEST) ? 1 : 0;
  // species densities at the ends: rho_s = x_s P / (s_s c_s^2)
  kp.rho_bc[0][0] = p->cl_in * p_in / (rc.s[0] * cs2);
  kp.rho_bc[0][1] = (1.0 - p->cl_in) * p_in / (rc.s[1] * cs2);
  kp.rho_bc[1][0] = p->cl_out * p_out / (rc.s[0] * cs2);
  kp.rho_bc[1][1] = (1.0 - p->cl_out) * p_out / (rc.s[1] * cs2);

  KBufs& kb = h->kb;
  kb.partials = reinterpret_cast<double*>(h->ws + L.partials);
  kb.endsum = reinterpret_cast<double*>(h->ws + L.endsum);
  kb.colsum = reinterpret_cast<double*>(h->ws + L.colsum);
  kb.strip = reinterpret_cast<double*>(h->ws + L.strip);
  kb.hist = reinterpret_cast<double*>(h->ws + L.hist);
  kb.counters = reinterpret_cast<unsigned*>(h->ws + L.counters);
  kb.status = kb.counters + (L.nxt + 1);
  kb.hist_cap = p->hist_cap;

  hipLaunchKernelGGL(k_zero_u32, dim3((L.nxt + 2 + 255) / 256), dim3(256), 0, h->stream, kb.counters, L.nxt + 2);
  const int igrid = (int)std::min<long long>(4096, ((long long)p->ny * L.pitch + 255) / 256);
  if (p->dtype == LBSEP_F64)
    hipLaunchKernelGGL(k_init<double>, dim3(igrid), dim3(kThreads), 0, h->stream, kp,
                       static_cast<double*>(h->f[0]), p_in, p_out, p->cl_in, p->cl_out);
  else
    hipLaunchKernelGGL(k_init<float>, dim3(igrid), dim3(kThreads), 0, h->stream, kp,
                       static_cast<float*>(h->f[0]), p_in, p_out, p->cl_in, p->cl_out);
  int rc_ = check_hip(hipGetLastError(), "init launch");
  if (rc_ == LBSEP_OK) rc_ = collide_loaded(h, 0);
  if (rc_ != LBSEP_OK) {
    delete h;
    return rc_;
  }
  *out = h;
  return LBSEP_OK;
}

int lbsep_step(lbsep_channel* h, int64_t nsteps) {
  if (!h) return fail(LBSEP_EINVAL, "channel is NULL");
  if (nsteps < 0) return fail(LBSEP_EINVAL, "nsteps must be >= 0");
  for (int64_t n = 0; n < nsteps; ++n) {
    const int nxt_buf = 1 - h->cur;
    sweep_any<true, false>(h, h->f[h->cur], h->f[nxt_buf], nullptr, nullptr, (long long)(h->t + 1));
    h->cur = nxt_buf;
    h->prev_pre = false;
    h->t += 1;
  }
  return check_hip(hipGetLastError(), "step launch");
}

int64_t lbsep_time(const lbsep_channel* h) { return h ? h->t : -1; }

int lbsep_read_cl(lbsep_channel* h, double* cl, double* cl_tilde, int32_t* x_min, double* profile) {
  if (!h) return fail(LBSEP_EINVAL, "channel is NULL");
  double rec[4];
  unsigned status = 0;
  const double* src = h->kb.hist + (h->t % h->kb.hist_cap) * 4;
  int rc = check_hip(hipMemcpyAsync(rec, src, sizeof(rec), hipMemcpyDeviceToHost, h->stream), "read_cl copy");
  if (rc) return rc;
  rc = check_hip(hipMemcpyAsync(&status, h->kb.status, sizeof(unsigned), hipMemcpyDeviceToHost, h->stream),
                 "read_cl status");
  if (rc) return rc;
  double* cs = nullptr;
  if (profile) {
    cs = new (std::nothrow) double[2 * (size_t)h->p.nx];
    if (!cs) return fail(LBSEP_EDEVICE, "out of host memory");
    rc = check_hip(hipMemcpy2DAsync(cs, h->p.nx * sizeof(double), h->kb.colsum, h->L.pitch * sizeof(double),
                                    h->p.nx * sizeof(double), 2, hipMemcpyDeviceToHost, h->stream),
                   "read_cl profile");
  }
  if (!rc) rc = check_hip(hipStreamSynchronize(h->stream), "read_cl sync");
  if (!rc && profile)
    for (int x = 0; x < h->p.nx; ++x) profile[x] = cs[x] / (cs[x] + cs[h->p.nx + x]);
  delete[] cs;
  if (rc) return rc;
  if (cl) *cl = rec[1];
  if (cl_tilde) *cl_tilde = rec[2];
  if (x_min) *x_min = (int32_t)rec[3];
  if (status & 1u) return fail(LBSEP_ENONFINITE, "non-finite or non-positive column density seen");
  return LBSEP_OK;
}

int lbsep_read_column_sums(lbsep_channel* h, double* host) {
  if (!h || !host) return fail(LBSEP_EINVAL, "NULL argument");
  int rc = check_hip(hipMemcpy2DAsync(host, h->p.nx * sizeof(double), h->kb.colsum, h->L.pitch * sizeof(double),
                                      h->p.nx * sizeof(double), 4, hipMemcpyDeviceToHost, h->stream),
                     "column sums copy");
  if (!rc) rc = check_hip(hipStreamSynchronize(h->stream), "column sums sync");
  return rc;
}

int lbsep_read_history(lbsep_channel* h, int64_t t0, int64_t count, double* host) {
  if (!h || (!host && count > 0) || count < 0) return fail(LBSEP_EINVAL, "bad argument");
  if (count == 0) return LBSEP_OK;
  const int64_t oldest = std::max<int64_t>(h->t_first, h->t - h->kb.hist_cap + 1);
  if (t0 < oldest || t0 + count - 1 > h->t)
    return fail(LBSEP_ERANGE, "history levels kept: " + std::to_string(oldest) + ".." + std::to_string(h->t));
  int64_t done = 0;
  while (done < count) {
    const int64_t slot = (t0 + done) % h->kb.hist_cap;
    const int64_t n = std::min<int64_t>(count - done, h->kb.hist_cap - slot);
    int rc = check_hip(hipMemcpyAsync(host + 4 * done, h->kb.hist + 4 * slot, n * 4 * sizeof(double),
                                      hipMemcpyDeviceToHost, h->stream),
                       "history copy");
    if (rc) return rc;
    done += n;
  }
  return check_hip(hipStreamSynchronize(h->stream), "history sync");
}

int lbsep_read_moments(lbsep_channel* h, double* host) {
  if (!h || !host) return fail(LBSEP_EINVAL, "NULL argument");
  int rc = eval_state(h, h->mom, nullptr);
  if (rc) return rc;
  rc = check_hip(hipMemcpyAsync(host, h->mom, 6ull * h->p.ny * h->p.nx * sizeof(double), hipMemcpyDeviceToHost,
                                h->stream),
                 "moments copy");
  if (!rc) rc = check_hip(hipStreamSynchronize(h->stream), "moments sync");
  return rc;
}

int lbsep_get_state(lbsep_channel* h, void* dev_dst) {
  if (!h || !dev_dst) return fail(LBSEP_EINVAL, "NULL argument");
  return eval_state(h, nullptr, dev_dst);
}

int lbsep_set_state(lbsep_channel* h, const void* dev_src, int64_t t) {
  if (!h || !dev_src) return fail(LBSEP_EINVAL, "NULL argument");
  if (t < 0) return fail(LBSEP_EINVAL, "t must be >= 0");
  const int grid = 2048;
  hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(256), 0, h->stream, h->kb.status, 1);
  if (h->p.dtype == LBSEP_F64)
    hipLaunchKernelGGL(k_copy_in<double>, dim3(grid), dim3(256), 0, h->stream, h->kp,
                       static_cast<const double*>(dev_src), static_cast<double*>(h->f[0]));
  else
    hipLaunchKernelGGL(k_copy_in<float>, dim3(grid), dim3(256), 0, h->stream, h->kp,
                       static_cast<const float*>(dev_src), static_cast<float*>(h->f[0]));
  int rc = check_hip(hipGetLastError(), "set_state copy");
  if (rc) return rc;
  return collide_loaded(h, t);
}

void lbsep_destroy(lbsep_channel* h) { delete h; }

}  // extern "C"
