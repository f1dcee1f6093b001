// lbsep: fused sweep kernel and host implementation of include/lbsep.h.
//
// One time step = one launch of k_sweep<Mode, /*PULL=*/true, /*EVAL=*/false, ...>
// (or of k_sweep_batch for several channels at once). For each node (x, j)
// the kernel
//   1. pulls the 18 post-collision populations of the previous step from its
//      neighbours (Eq. (MRT), pull form of the streaming),
//   2. replaces the wall-crossing pulls by diffuse-bounce-back (Eqs. (bot),
//      (bot2)) from its own post-collision populations,
//   3. on the inlet/outlet columns, extrapolates the populations entering from
//      the reservoir from the first and second inner layers and rescales the
//      node to the corrected extrapolated density (Eqs. (rho1), (rho2)),
//   4. computes moments (Eq. (rhou)), relaxation times (Eqs. (taos), (EQFrsp),
//      (taoq)) and collides both species (Eq. (MR)),
//   5. writes the 18 new post-collision populations, and
//   6. adds its species number density and x-momentum to FP64 column sums of
//      its tile. The reduction of those sums to C_l(x), CL and C~_l (Eqs. (C),
//      (CL), (Clline)) is pipelined across launches: the lead blocks of sweep t
//      reduce the tile sums of step t-1 to per-strip results, and one lead block
//      turns the strip results of step t-2 into the record (t-2, CL, C~_l,
//      x_min). The launch boundary orders producer and consumer, so the hot
//      path has no fences or atomics; the summation order is fixed. Reading
//      results first completes the last two levels (k_finalize).
//
// Storage modes (Mode<S, C, DEV>): FP64 stores f and computes in double.
// FP32 and FP16 store the deviation d = f - f0(x) from the rest equilibrium
// f0_si(x) = w_i alpha_si rho0_s(x) of a reference density linear in x
// (rho0(0) = rho_in, rho0(nx-1) = rho_out) and compute in float: the
// velocity, a small difference of O(1) populations, keeps the relative
// precision of the storage type. Streaming d across one column adds the
// constant -c_ix w_i alpha_si (d rho0 / dx); DBB and the extrapolation are the
// same formulas on d (f0 is at rest and linear in x); the collision uses
// rho - rho0 for the density terms.
//
// Layout in HBM (tile-blocked): each row is cut into blocks of 64 columns, and
// a block stores its nine directions one after the other, each as 64 nodes
// with the two species side by side (see pidx). A wavefront working on the 64
// columns of one block of one row reads and writes one contiguous 64-node run
// per direction, and the nine runs of a block are adjacent in memory.
// Two state buffers alternate; the one written last holds the post-collision
// state f'(t), the other the previous post-collision state f'(t-1) (or, right
// after init / set_state, the pre-collision state f(t)).
//
// Work decomposition, two tile shapes with the same arithmetic per node
// (chosen per channel, bitwise equal results); a block is W wavefronts (8 in
// FP32, 4 in FP64 and FP16):
//   lane pair per node (SPLIT): 32 columns x (W * rpt) rows; lanes 0-31 hold
//     species a and lanes 32-63 species b of the same 32 columns; the
//     relaxation-time work is split over the pair. Shortest chain per lane:
//     for channels that leave the GPU mostly idle.
//   one lane per node: 64 columns x (W * rpt) rows, both species in one lane;
//     fewest instructions per node: for channels that fill the GPU.
// Lead blocks come first: nendb blocks own the inlet and outlet columns in
// 64-row units (one unit per block of 4 wavefronts, two per block of 8; each
// unit needs the whole column's sum of the inner layers before it can rebuild
// its boundary nodes), then blocks that reduce one column strip per wavefront
// of the previous step, then one block that finishes the step before that.
// Tiles follow in plain row-major grid order (the hardware deals consecutive
// blocks to the 8 XCDs in turn, so the blocks in flight stay in one compact
// stretch of the state); on large channels their stores are non-temporal.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "lbsep.h"
#include "lbsep_device.h"
#include "lbsep_view.h"

namespace lbsep {
namespace {

constexpr int kTX = 64;         // columns per block (one wavefront across x)
constexpr int kTY = 4;          // wavefronts of the 256-thread units below
constexpr int kThreads = kTX * kTY;
// an inlet/outlet block's items: 4 lanes (species, inner layer) per row, 64 rows
constexpr int kEndThreads = 256;
constexpr int kMaxEnd = 32;     // end blocks per inlet/outlet column: ny <= 64 * kMaxEnd
constexpr unsigned kRowMajorTiles = 1u << 16;  // KParams::flags bit above the ABI flags

template <typename S, typename C, bool DEV>
struct Mode {
  using St = S;  // storage type of a population
  using Ct = C;  // arithmetic type
  using Pt = S __attribute__((ext_vector_type(2)));  // the two species of one population
  static constexpr bool kDev = DEV;
  static constexpr int kPsi = 0;  // FP64 wall function: the channel's choice, read at run time
};
using ModeF64 = Mode<double, double, false>;
using ModeF32 = Mode<float, float, true>;
using ModeF16 = Mode<_Float16, float, true>;

// Single-channel FP64 sweeps are compiled once per wall-function evaluation
// (PSI = 1: the series form, 2: the piecewise polynomials) and launched by the
// channel's choice, so that each holds only its own registers (with both
// behind a run-time switch the one-level FP64 sweep takes 176 VGPRs and two
// wavefronts per SIMD, against 126-159 and three). Batches and the two-level
// kernel read the choice at run time.
template <class MD, int PSI>
struct PsiMode : MD {
  static constexpr int kPsi = PSI;
};

// Wavefronts per block of the one-level sweep. FP32: 8, so that a tile of two
// rows per wavefront covers 16 rows and its column partial sums are half as
// many as with 4 (64-member table: 187.3 -> 184.8 us per step; 512 x 10240:
// 133.5 -> 132.0 us). FP64 and FP16 keep 4: their register counts (167 and 91
// VGPRs) leave room for 3 and 5 wavefronts per SIMD, which blocks of 8 would
// cut to 2 and 4 (the table: FP64 462 -> 658 us, FP16 148.8 -> 156.9 us).
template <class MD>
constexpr int kWaves = std::is_same<typename MD::St, float>::value ? 8 : 4;
constexpr int waves_of(int dtype) { return dtype == LBSEP_F32 ? 8 : 4; }

struct KParams {
  RelaxConsts rc;
  int nx, ny, pitch;
  int nxt, nrt, rpt;    // 64-column reduction strips, row tiles, rows per thread
  int ntx;              // 32-column tile strips
  int tiles;            // ntx * nrt
  int lead;             // lead blocks (multiple of 8) before the first tile
  int nend;             // 64-row units per inlet/outlet column
  int nendb;            // inlet/outlet blocks of a launch (one or two units each)
  long long row;        // elements per row of a state buffer: 18 * pitch
  unsigned flags;
  double r;             // DBB coefficient
  double rho_bc[2][2];  // [inlet/outlet][species] densities of Eq. (rho2)
  double cl_in;
  // deviation storage: rho0_s(x) = ref0[s] + slope[s] x, f0_si = wa[s][i] rho0_s
  double ref0[2], slope[2];
  double wa[2][9];
  double corr[2][9];    // -c_ix wa[s][i] slope[s]: streaming across one column
};

// Whether a sweep of mode MD on this channel evaluates the FP64 wall function
// from the piecewise polynomials.
template <class MD>
__device__ __forceinline__ bool psi_table(const KParams& kp) {
  return MD::kPsi == 0 ? kp.rc.psi_table != 0 : MD::kPsi == 2;
}

// Reduction buffers are double-buffered by the parity of the time level.
struct KBufs {
  double* partials;    // [2][4][nrt][pitch] per row-tile column sums
  double* endsum;      // [2][2][kMaxEnd][4] inlet / outlet column sums per end block
  double* colsum;      // [4][pitch] column sums of the last reduced level
  double* strip;       // [2][nxt][4] (min C_l, argmin, sum (C_l - C_in), bad)
  double* hist;        // [hist_cap][4] (t, CL, C~_l, x_min)
  unsigned* status;    // [1] bit 0: non-finite or non-positive column density seen
  long long hist_cap;
  long long part_stride;   // elements of one partials buffer: 4 * nrt * pitch
};

// State buffer layout: row j holds pitch / 64 blocks of 64 columns; block b
// holds direction 0, then 1, ... 8, each as 64 consecutive nodes with the two
// species of a node side by side:
//   element j * 18 pitch + ((b * 9 + i) * 64 + (x mod 64)) * 2 + s,  b = x / 64.
// One lane holding both species of a node moves a direction with a single
// 2-element access that stays aligned whatever the +-1 column shift; the
// nine direction runs and the write-back of a block are contiguous.
// element offset of (s = 0, i = 0) of column x inside its row
__device__ __forceinline__ unsigned col_off(int x) {
  return (((unsigned)x >> 6) * 576u + ((unsigned)x & 63u)) * 2u;
}
__device__ __forceinline__ long long pidx(const KParams& kp, int s, int i, int j, int x) {
  return (long long)j * kp.row + i * 128 + s + col_off(x);
}

// Population (s, i) at (j, x) of a state buffer as a base for (row, direction,
// species), wave-uniform where j is, plus a 32-bit byte offset of the column
// inside the row: loads and stores then address through a scalar base and one
// of three column offsets (x - 1, x, x + 1).
template <typename S>
__device__ __forceinline__ S* pop_at(const KParams& kp, S* base, int s, int i, int j, int x) {
  S* rw = base + ((long long)j * kp.row + (i * 128 + s));
  return reinterpret_cast<S*>(reinterpret_cast<char*>(rw) + col_off(x) * (unsigned)sizeof(S));
}
template <typename S>
__device__ __forceinline__ const S* pop_at(const KParams& kp, const S* base, int s, int i, int j, int x) {
  const S* rw = base + ((long long)j * kp.row + (i * 128 + s));
  return reinterpret_cast<const S*>(reinterpret_cast<const char*>(rw) + col_off(x) * (unsigned)sizeof(S));
}
// Both species of population i at (j, x).
template <class MD>
__device__ __forceinline__ typename MD::Pt* pair_at(const KParams& kp, typename MD::St* base, int i, int j, int x) {
  return reinterpret_cast<typename MD::Pt*>(pop_at(kp, base, 0, i, j, x));
}
template <class MD>
__device__ __forceinline__ const typename MD::Pt* pair_at(const KParams& kp, const typename MD::St* base, int i, int j,
                                                          int x) {
  return reinterpret_cast<const typename MD::Pt*>(pop_at(kp, base, 0, i, j, x));
}

// Entry s of a per-species parameter pair: an index, or (SEL) a select
// between the two entries.
template <bool SEL>
__device__ __forceinline__ double species_param(const double (&v)[2], int s) {
  return SEL ? (s ? v[1] : v[0]) : v[s];
}

__device__ __forceinline__ double ref_rho(const KParams& kp, int s, int x) {
  return kp.ref0[s] + kp.slope[s] * double(x);
}

template <typename T>
__device__ __forceinline__ T sum9(const T f[9]) {
  return ((f[0] + f[1]) + (f[2] + f[3])) + ((f[4] + f[5]) + (f[6] + f[7])) + f[8];
}

// Rounding in the deviation storage modes. Near a steady state a node's
// populations change by far less than their own rounding unit per step, so
// a rounding that depends only on the value's position on the float grid
// returns the same residual at every step: a frozen error that the slow
// hydrodynamic modes (decay rates down to 1e-5 per step) amplify by their
// inverse decay rate. Two places would do that:
//   - streaming across a column adds the constant c_i of the reference state
//     (add_stream_corr) to a float d: fl(d + c) rounds c to the grid of d,
//     the same error at every node whose d lies in the same binade, a
//     systematic error of about ulp(d) / |c| (1e-5 on the parametric table)
//     in the reference pressure force (measured: a CL drift of about 1e-9 per
//     step in FP32 against FP64, against 1e-10 for a 1e-7 perturbation of an
//     FP64 run);
//   - the binary16 store of a post-collision value rounds to a grid 2^13
//     times coarser than the float arithmetic (dither_species).
// Both add u ulp(v) before rounding, u uniform on [-1/2, 1/2) and ulp(v) the
// rounding unit at v, which makes the expected result the exact one
// (stochastic rounding). u comes from a counter-based generator keyed by the
// node, the time level, the species and the direction, so every kernel that
// forms a level's values forms the same bits, and runs stay bitwise
// reproducible.
__device__ __forceinline__ unsigned dither_seed(int x, int j, long long t) {
  unsigned h = (unsigned)x * 0x9E3779B1u ^ (unsigned)j * 0x85EBCA77u ^ (unsigned)t * 0xC2B2AE3Du ^
               (unsigned)((unsigned long long)t >> 32) * 0x27D4EB2Fu;
  h = h * 747796405u + 2891336453u;  // PCG step and RXS-M-XS output permutation
  h = ((h >> ((h >> 28u) + 4u)) ^ h) * 277803737u;
  return (h >> 22u) ^ h;
}

// The node's generator is a linear congruential sequence r' = a r + c from
// its seed; each state gives two 16-bit uniforms. Sub-streams: the streaming
// correction of species 0 / 1 uses states 1-3 / 4-6, the binary16 store of
// species 0 / 1 states 7-11 / 12-16; a sub-stream is entered by jumping
// ahead (r_k = A_k r + C_k, one multiply-add).
constexpr unsigned kLcgA = 1664525u, kLcgC = 1013904223u;
struct LcgJump {
  unsigned a, c;
};
constexpr LcgJump lcg_jump(int k) {
  unsigned a = 1u, c = 0u;
  for (int i = 0; i < k; ++i) {
    a = a * kLcgA;
    c = c * kLcgA + kLcgC;
  }
  return {a, c};
}
template <int K>
__device__ __forceinline__ unsigned lcg_at(unsigned seed) {
  constexpr LcgJump J = lcg_jump(K);
  return J.a * seed + J.c;
}

// Uniforms on (-1/2, 1/2) from the high and low halves of a generator state
// (16 bits each, centred: a rounding bias of at most 2^-17 of a unit remains).
__device__ __forceinline__ float dither_hi(unsigned r) { return float(r >> 16) * 0x1p-16f - (0.5f - 0x1p-17f); }
__device__ __forceinline__ float dither_lo(unsigned r) { return float(r & 0xffffu) * 0x1p-16f - (0.5f - 0x1p-17f); }

// Unit in the last place of the storage type S at the float value v (0 for
// zero and float subnormals).
template <typename S>
__device__ __forceinline__ float storage_ulp(float v) {
  const float p2 = __uint_as_float(__float_as_uint(v) & 0x7f800000u);  // 2^floor(log2 |v|)
  if constexpr (std::is_same<S, float>::value)
    return p2 * 0x1p-23f;
  else
    return fmaxf(p2 * 0x1p-10f, 0x1p-24f);  // binary16: 10 fraction bits, subnormal step 2^-24
}

// Streaming correction of species s at node (x, j), level t (deviation
// modes): the populations pulled across a column (c_ix != 0: directions 1,
// 3, 5, 6, 7, 8) gain corr = -c_ix w_i alpha_si d rho0/dx, added with
// stochastic rounding.
template <class MD>
__device__ __forceinline__ void add_stream_corr(const KParams& kp, int x, int j, long long t, int s,
                                                typename MD::Ct f[9]) {
  static_assert(MD::kDev, "only deviations are corrected");
  const unsigned seed = dither_seed(x, j, t);
  const unsigned r1 = s ? lcg_at<4>(seed) : lcg_at<1>(seed);
  const unsigned r2 = r1 * kLcgA + kLcgC;
  const unsigned r3 = r2 * kLcgA + kLcgC;
  const float u[6] = {dither_hi(r1), dither_lo(r1), dither_hi(r2), dither_lo(r2), dither_hi(r3), dither_lo(r3)};
  const int dir[6] = {1, 3, 5, 6, 7, 8};
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    const int i = dir[k];
    f[i] += __builtin_fmaf(u[k], storage_ulp<float>(f[i]), float(kp.corr[s][i]));
  }
}

// Stochastic rounding of the binary16 store: species s of node (x, j) at
// level t, post-collision.
template <class MD>
__device__ __forceinline__ void dither_species(typename MD::Ct f[9], int x, int j, long long t, int s) {
  static_assert(MD::kDev, "only the deviation storage modes are dithered");
  const unsigned seed = dither_seed(x, j, t);
  unsigned r = s ? lcg_at<12>(seed) : lcg_at<7>(seed);
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    const float u = (i & 1) ? dither_lo(r) : dither_hi(r);
    if (i & 1) r = r * kLcgA + kLcgC;
    f[i] += u * storage_ulp<typename MD::St>(f[i]);
    // the float value itself, rounded once more to binary16 by the store: the
    // compiler must not fuse this addition with that conversion on some
    // paths only (a single rounding there would give other bits than the
    // same level formed by another kernel)
    asm volatile("" : "+v"(f[i]));
  }
}

// Whether the post-collision values of mode MD are dithered before the store.
template <class MD>
constexpr bool kDitherStore = MD::kDev && !std::is_same<typename MD::St, float>::value;

// Pre-collision populations (deviations in the FP32/FP16 modes) of species s
// at node (x, j) at the new time level.
// PULL: streamed from the post-collision state in src, with DBB on wall rows.
// !PULL: read in place (src already holds a pre-collision state).
// On the inlet/outlet columns the directions that would come from outside the
// channel are loaded from the node itself (kept in range) and replaced by the
// caller.
template <class MD, bool PULL>
__device__ __forceinline__ void gather1(const KParams& kp, const typename MD::St* __restrict__ src, int s, int x,
                                        int j, long long t, typename MD::Ct f[9]) {
  using C = typename MD::Ct;
  if (!PULL) {
#pragma unroll
    for (int i = 0; i < 9; ++i) f[i] = C(*pop_at(kp, src, s, i, j, x));
    return;
  }
  int xm = x - 1, xp = x + 1, jm = j - 1, jp = j + 1;
  if (kp.flags & LBSEP_PERIODIC_X) {
    if (xm < 0) xm += kp.nx;
    if (xp >= kp.nx) xp -= kp.nx;
  } else {
    if (xm < 0) xm = 0;
    if (xp >= kp.nx) xp = kp.nx - 1;
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
  for (int i = 0; i < 9; ++i) f[i] = C(*pop_at(kp, src, s, i, sy[i], sx[i]));
  if constexpr (MD::kDev) add_stream_corr<MD>(kp, x, j, t, s, f);
  if (bot || top) {
    // Eqs. (bot)/(bot2): the populations that would come from outside the
    // channel are r f^eq(rho_w, u_w = 0) + (1 - r) f'_opposite at the same node;
    // rho_w makes the returned mass equal the leaving mass F, which puts the
    // shares 4/6, 1/6, 1/6 of F on the axis and the two diagonal directions.
    // The rest equilibrium is a fixed point of this map, so deviations obey it too.
    // (constant array indices in each branch keep f in registers)
    const int o0 = bot ? 4 : 2, o1 = bot ? 7 : 5, o2 = bot ? 8 : 6;  // leaving
    const C l0 = C(*pop_at(kp, src, s, o0, j, x));
    const C l1 = C(*pop_at(kp, src, s, o1, j, x));
    const C l2 = C(*pop_at(kp, src, s, o2, j, x));
    C v0, v1, v2;
    dbb_shares<C>(C(kp.r), l0, l1, l2, v0, v1, v2);
    if (bot) {  // returning 2, 5, 6
      f[2] = v0;
      f[5] = v1;
      f[6] = v2;
    } else {    // returning 4, 7, 8
      f[4] = v0;
      f[7] = v1;
      f[8] = v2;
    }
  }
}

// DBB of gather1 for both species of a wall node (bot: the bottom wall):
// w0, w1, w2 are the node's own leaving pairs (directions 4, 7, 8 at the
// bottom, 2, 5, 6 at the top); the returning directions of fa, fb are replaced.
template <class MD>
__device__ __forceinline__ void dbb_pair(const KParams& kp, bool bot, typename MD::Pt w0, typename MD::Pt w1,
                                         typename MD::Pt w2, typename MD::Ct fa[9], typename MD::Ct fb[9]) {
  using C = typename MD::Ct;
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    C v0, v1, v2;
    dbb_shares<C>(C(kp.r), C(w0[s]), C(w1[s]), C(w2[s]), v0, v1, v2);
    C* f = s ? fb : fa;
    if (bot) {
      f[2] = v0;
      f[5] = v1;
      f[6] = v2;
    } else {
      f[4] = v0;
      f[7] = v1;
      f[8] = v2;
    }
  }
}

// Both species at node (x, j), one 2-element access per direction: the same
// values as gather1 for s = 0 and s = 1.
template <class MD, bool PULL>
__device__ __forceinline__ void gather_pair(const KParams& kp, const typename MD::St* __restrict__ src, int x, int j,
                                            long long t, typename MD::Ct fa[9], typename MD::Ct fb[9]) {
  using C = typename MD::Ct;
  if (!PULL) {
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      const typename MD::Pt v = *pair_at<MD>(kp, src, i, j, x);
      fa[i] = C(v[0]);
      fb[i] = C(v[1]);
    }
    return;
  }
  int xm = x - 1, xp = x + 1, jm = j - 1, jp = j + 1;
  if (kp.flags & LBSEP_PERIODIC_X) {
    if (xm < 0) xm += kp.nx;
    if (xp >= kp.nx) xp -= kp.nx;
  } else {
    if (xm < 0) xm = 0;
    if (xp >= kp.nx) xp = kp.nx - 1;
  }
  bool bot = false, top = false;
  if (kp.flags & LBSEP_PERIODIC_Y) {
    if (jm < 0) jm += kp.ny;
    if (jp >= kp.ny) jp -= kp.ny;
  } else {
    bot = (j == 0);
    top = (j == kp.ny - 1);
    if (bot) jm = j;
    if (top) jp = j;
  }
  const int sx[9] = {x, xm, x, xp, x, xm, xp, xp, xm};
  const int sy[9] = {j, j, jm, j, jp, jm, jm, jp, jp};
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    const typename MD::Pt v = *pair_at<MD>(kp, src, i, sy[i], sx[i]);
    fa[i] = C(v[0]);
    fb[i] = C(v[1]);
  }
  if constexpr (MD::kDev) {
    add_stream_corr<MD>(kp, x, j, t, 0, fa);
    add_stream_corr<MD>(kp, x, j, t, 1, fb);
  }
  if (bot || top) {  // the DBB map of gather1, both species
    const int o0 = bot ? 4 : 2, o1 = bot ? 7 : 5, o2 = bot ? 8 : 6;
    const typename MD::Pt w0 = *pair_at<MD>(kp, src, o0, j, x);
    const typename MD::Pt w1 = *pair_at<MD>(kp, src, o1, j, x);
    const typename MD::Pt w2 = *pair_at<MD>(kp, src, o2, j, x);
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      C v0, v1, v2;
      dbb_shares<C>(C(kp.r), C(w0[s]), C(w1[s]), C(w2[s]), v0, v1, v2);
      C* f = s ? fb : fa;
      if (bot) {
        f[2] = v0;
        f[5] = v1;
        f[6] = v2;
      } else {
        f[4] = v0;
        f[7] = v1;
        f[8] = v2;
      }
    }
  }
}

// Rebuilt pre-collision node of species s on the inlet (e = 0) or outlet
// (e = 1) column, Eqs. (rho1), (rho2): f holds the node's pulled populations,
// g1 / g2 those of the first / second inner layer. The populations entering
// from the reservoir are extrapolated, then the node is rescaled to
// kappa rho'(j) with rho' = 2 rho(l1, j) - rho(l2, j).
// kap = kappa; km1 = kappa - 1 (used by the deviation modes).
template <class MD>
__device__ __forceinline__ void end_rebuild(const KParams& kp, int e, int s, int col, double kap, double km1,
                                            const typename MD::Ct g1[9], const typename MD::Ct g2[9],
                                            typename MD::Ct f[9]) {
  using C = typename MD::Ct;
  if (e == 0) {  // entering at the inlet: c_x = +1
    f[1] = C(2) * g1[1] - g2[1];
    f[5] = C(2) * g1[5] - g2[5];
    f[8] = C(2) * g1[8] - g2[8];
  } else {       // entering at the outlet: c_x = -1
    f[3] = C(2) * g1[3] - g2[3];
    f[6] = C(2) * g1[6] - g2[6];
    f[7] = C(2) * g1[7] - g2[7];
  }
  const C rp = C(2) * sum9(g1) - sum9(g2);  // rho' (deviation modes: rho' - rho0(col))
  if (!MD::kDev) {
    const C scale = (C(kap) * rp) / sum9(f);
#pragma unroll
    for (int i = 0; i < 9; ++i) f[i] *= scale;
  } else {
    // f -> S f with S - 1 = ((kappa - 1) rho0 + kappa d rho' - d rho_node) / rho_node
    const double r0d = ref_rho(kp, s, col);
    const C r0 = C(r0d);
    const C dn = sum9(f);
    const C sm1 = (C(km1 * r0d) + C(kap) * rp - dn) / (r0 + dn);
#pragma unroll
    for (int i = 0; i < 9; ++i) f[i] += sm1 * (f[i] + C(kp.wa[s][i] * r0d));
  }
}

// What the collision of a node needs from its moments and relaxation times.
template <typename C>
struct NodeState {
  C ca, cb;        // conserved density parts (rho, or rho - rho0 for deviations)
  C rho_a, rho_b;  // species densities
  C ux, uy;        // mixture velocity
  C ts, tq, h2;    // tau_s, tau_q and 1 / (2 tau_d)
};

// Moments and relaxation times of one node by one lane holding both species
// (fa, fb: populations, deviations in the FP32/FP16 modes); (STEP) adds the
// node to acc = (n_a, n_b, rho_a u_ax, rho_b u_bx), (EVAL) writes the outputs.
template <class MD, bool EVAL>
__device__ __forceinline__ NodeState<typename MD::Ct> node_moments(const KParams& kp, int x, int j,
                                                                   const typename MD::Ct fa[9],
                                                                   const typename MD::Ct fb[9],
                                                                   double* __restrict__ mom,
                                                                   typename MD::St* __restrict__ fraw,
                                                                   double* __restrict__ ffull, double acc[4]) {
  using C = typename MD::Ct;
  using E = E1Traits<C>;
  const C ca = sum9(fa);  // rho_a, or rho_a - rho0_a(x)
  const C cb = sum9(fb);
  const double r0a = MD::kDev ? ref_rho(kp, 0, x) : 0.0;
  const double r0b = MD::kDev ? ref_rho(kp, 1, x) : 0.0;
  const double ra_d = MD::kDev ? r0a + double(ca) : double(ca);
  const double rb_d = MD::kDev ? r0b + double(cb) : double(cb);
  const C rho_a = MD::kDev ? C(ra_d) : ca;
  const C rho_b = MD::kDev ? C(rb_d) : cb;
  const C jxa = (fa[1] - fa[3]) + (fa[5] - fa[6]) + (fa[8] - fa[7]);
  const C jya = (fa[2] - fa[4]) + (fa[5] + fa[6]) - (fa[7] + fa[8]);
  const C jxb = (fb[1] - fb[3]) + (fb[5] - fb[6]) + (fb[8] - fb[7]);
  const C jyb = (fb[2] - fb[4]) + (fb[5] + fb[6]) - (fb[7] + fb[8]);
  const C inv_rho = E::rcp(rho_a + rho_b);
  const C ux = (jxa + jxb) * inv_rho;  // mixture velocity, Eq. (rhou)
  const C uy = (jya + jyb) * inv_rho;
  C ts, td, tq;
  relaxation_times<C>(kp.rc, j, rho_a, rho_b, ts, td, tq, psi_table<MD>(kp));
  // species momentum of Eq. (rhou): rho_s u_s = (1 - 1/(2 tau_d)) j_s + rho_s u / (2 tau_d)
  const C h2 = C(0.5) * E::rcp(td);
  const C g = C(1) - h2;
  const C pxa = g * jxa + rho_a * ux * h2;
  const C pxb = g * jxb + rho_b * ux * h2;
  const NodeState<C> st{ca, cb, rho_a, rho_b, ux, uy, ts, tq, h2};
  if (EVAL) {
    const long long n = (long long)kp.nx * kp.ny;
    const long long o = (long long)j * kp.nx + x;
    if (mom) {
      const C pya = g * jya + rho_a * uy * h2;
      const C pyb = g * jyb + rho_b * uy * h2;
      mom[o] = ra_d;
      mom[n + o] = rb_d;
      mom[2 * n + o] = double(pxa / rho_a);
      mom[3 * n + o] = double(pya / rho_a);
      mom[4 * n + o] = double(pxb / rho_b);
      mom[5 * n + o] = double(pyb / rho_b);
    }
    if (fraw) {
#pragma unroll
      for (int i = 0; i < 9; ++i) {
        fraw[i * n + o] = typename MD::St(fa[i]);
        fraw[(9 + i) * n + o] = typename MD::St(fb[i]);
      }
    }
    if (ffull) {
#pragma unroll
      for (int i = 0; i < 9; ++i) {
        ffull[i * n + o] = double(fa[i]) + (MD::kDev ? kp.wa[0][i] * r0a : 0.0);
        ffull[(9 + i) * n + o] = double(fb[i]) + (MD::kDev ? kp.wa[1][i] * r0b : 0.0);
      }
    }
    acc[2] += double(pxa);  // the momentum sums, as a step adds them
    acc[3] += double(pxb);
    return st;
  }
  acc[0] += ra_d * kp.rc.inv_m[0];
  acc[1] += rb_d * kp.rc.inv_m[1];
  acc[2] += double(pxa);
  acc[3] += double(pxb);
  return st;
}

// Collision of both species of one node (moment state from node_moments), in
// place.
// The post-collision values of level t at node (x, j) are dithered when the
// storage type is binary16 (dither_species).
template <class MD>
__device__ __forceinline__ void node_collide_only(const KParams& kp, int x, int j, long long t, typename MD::Ct fa[9],
                                                  typename MD::Ct fb[9], const NodeState<typename MD::Ct>& st) {
  using C = typename MD::Ct;
  using E = E1Traits<C>;
  C we, weps;
  const C ws = E::rcp(st.ts);
  if (kp.rc.bgk) {
    we = weps = ws;
  } else {
    we = C(1.0 / 1.1);    // tau_e = 1.1 (Sec. 3.3)
    weps = C(1.0 / 1.2);  // tau_eps = 1.2
  }
  const C wd = C(2) * st.h2, wq = E::rcp(st.tq);
  collide_species<C>(fa, st.ca, st.rho_a, st.ux, st.uy, C(kp.rc.s[0]), we, weps, wd, wq, ws);
  collide_species<C>(fb, st.cb, st.rho_b, st.ux, st.uy, C(kp.rc.s[1]), we, weps, wd, wq, ws);
  if constexpr (kDitherStore<MD>) {
    dither_species<MD>(fa, x, j, t, 0);
    dither_species<MD>(fb, x, j, t, 1);
  }
}

// The post-collision pair of each direction of node (x, j) to dst.
template <class MD, bool NT>
__device__ __forceinline__ void node_store(const KParams& kp, int x, int j, const typename MD::Ct fa[9],
                                           const typename MD::Ct fb[9], typename MD::St* __restrict__ dst) {
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    typename MD::Pt v;
    v[0] = typename MD::St(fa[i]);
    v[1] = typename MD::St(fb[i]);
    if (NT)  // the next read of these lines is a whole sweep away: bypass the caches
      __builtin_nontemporal_store(v, pair_at<MD>(kp, dst, i, j, x));
    else
      *pair_at<MD>(kp, dst, i, j, x) = v;
  }
}

// Species s of node (x, j) to the dense FP64 array out[2][9][ny][nx] (a
// recording step of an FP64 channel: the populations themselves).
template <class MD>
__device__ __forceinline__ void dense_out(const KParams& kp, int x, int j, int s, const typename MD::Ct f[9],
                                          double* __restrict__ out) {
  static_assert(!MD::kDev, "recording steps hold plain populations");
  const long long n = (long long)kp.nx * kp.ny, o = (long long)j * kp.nx + x;
#pragma unroll
  for (int i = 0; i < 9; ++i) out[(9 * s + i) * n + o] = double(f[i]);
}

// node_moments, then (STEP) the collision and the store. REC (a recording
// step): ffull receives the pulled populations and fpost the post-collision
// ones, both dense.
template <class MD, bool EVAL, bool NT = false, bool REC = false>
__device__ __forceinline__ void process_node(const KParams& kp, int x, int j, long long t, typename MD::Ct fa[9],
                                             typename MD::Ct fb[9], typename MD::St* __restrict__ dst,
                                             double* __restrict__ mom, typename MD::St* __restrict__ fraw,
                                             double* __restrict__ ffull, double acc[4],
                                             double* __restrict__ fpost = nullptr) {
  const NodeState<typename MD::Ct> st = node_moments<MD, EVAL>(kp, x, j, fa, fb, mom, fraw, ffull, acc);
  if (!EVAL) {
    if constexpr (REC) {
      dense_out<MD>(kp, x, j, 0, fa, ffull);
      dense_out<MD>(kp, x, j, 1, fb, ffull);
    }
    node_collide_only<MD>(kp, x, j, t, fa, fb, st);
    node_store<MD, NT>(kp, x, j, fa, fb, dst);
    if constexpr (REC) {
      dense_out<MD>(kp, x, j, 0, fa, fpost);
      dense_out<MD>(kp, x, j, 1, fb, fpost);
    }
  }
}

// Moments, relaxation times and (STEP) collision + store or (EVAL) output of
// one node by a lane pair: this lane holds species s (f: its 9 populations,
// deviations in the FP32/FP16 modes), the partner lane (lane ^ XOR) the other
// species. Every lane of the wave must call this (it swaps values across the
// pair); lanes with active == false only feed the swaps. acc receives this
// species' (n_s, rho_s u_sx) in double. STORE == false leaves the
// post-collision populations in f instead of storing them to dst; SEL picks
// the per-species parameters by selects (kernels in which a dynamic index
// would move the parameter block to scratch memory); REC as in process_node.
template <class MD, bool EVAL, int XOR, bool STORE = true, bool SEL = false, bool REC = false>
__device__ __forceinline__ void process_pair(const KParams& kp, int x, int j, long long t, int s, bool active,
                                             typename MD::Ct f[9], typename MD::St* __restrict__ dst,
                                             double* __restrict__ mom, typename MD::St* __restrict__ fraw,
                                             double* __restrict__ ffull, double acc[2],
                                             double* __restrict__ fpost = nullptr) {
  using C = typename MD::Ct;
  using E = E1Traits<C>;
  if (!active) {
#pragma unroll
    for (int i = 0; i < 9; ++i) f[i] = MD::kDev ? C(0) : C(0.1);  // finite filler for the swaps
  }
  const C c_own = sum9(f);  // rho_s, or rho_s - rho0_s(x)
  const double r0 = MD::kDev ? species_param<SEL>(kp.ref0, s) + species_param<SEL>(kp.slope, s) * double(x) : 0.0;
  const double r_own = MD::kDev ? r0 + double(c_own) : double(c_own);
  const C rho_own = MD::kDev ? C(r_own) : c_own;
  const C jx = (f[1] - f[3]) + (f[5] - f[6]) + (f[8] - f[7]);
  const C jy = (f[2] - f[4]) + (f[5] + f[6]) - (f[7] + f[8]);
  const C rho_oth = lane_xor(rho_own, XOR);
  const C jx_oth = lane_xor(jx, XOR);
  const C jy_oth = lane_xor(jy, XOR);
  const C rho_a = s ? rho_oth : rho_own;
  const C rho_b = s ? rho_own : rho_oth;
  const C jxa = s ? jx_oth : jx, jxb = s ? jx : jx_oth;
  const C jya = s ? jy_oth : jy, jyb = s ? jy : jy_oth;
  const C inv_rho = E::rcp(rho_a + rho_b);
  const C ux = (jxa + jxb) * inv_rho;  // mixture velocity, Eq. (rhou)
  const C uy = (jya + jyb) * inv_rho;
  C ts, td, tq;
  relaxation_times_pair<C, XOR>(kp.rc, j, s, rho_a, rho_b, ts, td, tq, psi_table<MD>(kp));
  // species momentum of Eq. (rhou): rho_s u_s = (1 - 1/(2 tau_d)) j_s + rho_s u / (2 tau_d)
  const C h2 = C(0.5) * E::rcp(td);
  const C g = C(1) - h2;
  const C px = g * jx + rho_own * ux * h2;
  if (EVAL) {
    if (!active) return;
    const long long n = (long long)kp.nx * kp.ny;
    const long long o = (long long)j * kp.nx + x;
    if (mom) {
      const C py = g * jy + rho_own * uy * h2;
      mom[s * n + o] = r_own;
      mom[(2 + 2 * s) * n + o] = double(px / rho_own);
      mom[(3 + 2 * s) * n + o] = double(py / rho_own);
    }
    if (fraw) {
#pragma unroll
      for (int i = 0; i < 9; ++i) fraw[(9 * s + i) * n + o] = typename MD::St(f[i]);
    }
    if (ffull) {
#pragma unroll
      for (int i = 0; i < 9; ++i) ffull[(9 * s + i) * n + o] = double(f[i]) + (MD::kDev ? kp.wa[s][i] * r0 : 0.0);
    }
    acc[1] += double(px);  // the momentum sum, as a step adds it
    return;
  }
  C we, weps;
  const C ws = E::rcp(ts);
  if (kp.rc.bgk) {
    we = weps = ws;
  } else {
    we = C(1.0 / 1.1);    // tau_e = 1.1 (Sec. 3.3)
    weps = C(1.0 / 1.2);  // tau_eps = 1.2
  }
  const C wd = C(2) * h2, wq = E::rcp(tq);
  if constexpr (REC) {
    if (active) dense_out<MD>(kp, x, j, s, f, ffull);
  }
  collide_species<C>(f, c_own, rho_own, ux, uy, C(species_param<SEL>(kp.rc.s, s)), we, weps, wd, wq, ws);
  if (!active) return;
  if constexpr (kDitherStore<MD>) dither_species<MD>(f, x, j, t, s);
  if constexpr (REC) dense_out<MD>(kp, x, j, s, f, fpost);
  acc[0] += r_own * species_param<SEL>(kp.rc.inv_m, s);
  acc[1] += double(px);
  if (!STORE) return;
#pragma unroll
  for (int i = 0; i < 9; ++i) *pop_at(kp, dst, s, i, j, x) = typename MD::St(f[i]);
}

// Column sums of one strip (64 columns) of level `step`: add the row-tile
// partials (the inlet/outlet columns come from their own blocks), store them,
// and reduce the strip to (min C_l, its column, sum (C_l - C_in), bad flag).
// par: the level's slot in the reduction buffers; nrt, stride: row tiles and
// slot size of the partials; nq: the sums carried (2: the densities, as
// one-level launches write; 4: also the momenta). Run by one wavefront (lane =
// column), which keeps the sums of its column: each is added in row-tile order.
__device__ __forceinline__ void strip_reduce(const KParams& kp, const KBufs& kb, int bx, long long step, int par,
                                             int nrt, long long stride, int nq, bool store_cols = true) {
  const int lane = threadIdx.x & (kTX - 1);
  const int x = bx * kTX + lane;
  const bool px = kp.flags & LBSEP_PERIODIC_X;
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  if (x < kp.nx) {
    if (!px && (x == 0 || x == kp.nx - 1)) {
      const double* p = kb.endsum + (par * 2 + (x == 0 ? 0 : 1)) * kMaxEnd * 4;
      for (int b = 0; b < kp.nend; ++b) {
#pragma unroll
        for (int q = 0; q < 4; ++q)
          if (q < nq) v[q] += p[b * 4 + q];
      }
    } else {
      // loads issued up to 32 at a time (the partials were just written by
      // other XCDs, so each one is a trip past this XCD's L2)
      const double* p = kb.partials + par * stride + x;
      for (int b0 = 0; b0 < nrt; b0 += 8) {
        double w[4][8];
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
          for (int k = 0; k < 8; ++k)
            w[q][k] = q < nq && b0 + k < nrt ? p[((long long)q * nrt + b0 + k) * kp.pitch] : 0.0;
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
          for (int k = 0; k < 8; ++k)
            if (q < nq && b0 + k < nrt) v[q] += w[q][k];
      }
    }
    if (store_cols) {
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (q < nq) kb.colsum[(long long)q * kp.pitch + x] = v[q];
    }
  }
  double cl = 1e300, dev = 0.0, arg = 1e300;
  double bad = 0.0;
  if (x < kp.nx) {
    const double na = v[0], nb = v[1];
    cl = na / (na + nb);
    dev = cl - kp.cl_in;
    arg = double(x);
    const bool ok = (na > 0.0) && (nb > 0.0) && isfinite(na + nb);
    bad = ok ? 0.0 : 1.0;
    if (!ok) cl = -1e300;  // keep a bad column visible in the minimum
  }
  // wavefront tree reductions: min (ties -> smaller x), sum, max
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const double ocl = lane_xor(cl, off);
    const double oarg = lane_xor(arg, off);
    const double odev = lane_xor(dev, off);
    const double obad = lane_xor(bad, off);
    if (ocl < cl || (ocl == cl && oarg < arg)) {
      cl = ocl;
      arg = oarg;
    }
    dev += odev;
    bad = fmax(bad, obad);
  }
  if (lane == 0) {
    double* st = kb.strip + ((long long)par * kp.nxt + bx) * 4;
    st[0] = cl;
    st[1] = arg;
    st[2] = dev;
    st[3] = bad;
  }
}

// Strip-reduction blocks of a launch: each wavefront of a block reduces one
// strip.
__host__ __device__ constexpr int strip_blocks(int nxt, int waves) { return (nxt + waves - 1) / waves; }

// The momentum column sums (quantities 2, 3) of one strip from the partials
// of slot par (written by an evaluation sweep), added in row-tile order and
// stored to colsum. One wavefront (lane = column).
__device__ __forceinline__ void jsum_reduce(const KParams& kp, const KBufs& kb, int bx, int par) {
  const int x = bx * kTX + int(threadIdx.x & (kTX - 1));
  if (x >= kp.nx) return;
  double v[2] = {0.0, 0.0};
  if (!(kp.flags & LBSEP_PERIODIC_X) && (x == 0 || x == kp.nx - 1)) {
    const double* p = kb.endsum + (par * 2 + (x == 0 ? 0 : 1)) * kMaxEnd * 4;
    for (int b = 0; b < kp.nend; ++b) {
      v[0] += p[b * 4 + 2];
      v[1] += p[b * 4 + 3];
    }
  } else {
    const double* p = kb.partials + par * kb.part_stride + x;
    for (int b = 0; b < kp.nrt; ++b) {
      v[0] += p[((long long)2 * kp.nrt + b) * kp.pitch];
      v[1] += p[((long long)3 * kp.nrt + b) * kp.pitch];
    }
  }
  kb.colsum[2LL * kp.pitch + x] = v[0];
  kb.colsum[3LL * kp.pitch + x] = v[1];
}

// Record of level `step` from its strip results (slot par): CL (Eq. (CL)),
// C~_l (Eq. (Clline)) and the column of the smallest C_l. One wavefront.
__device__ __forceinline__ void global_reduce(const KParams& kp, const KBufs& kb, long long step, int par) {
  const int lane = threadIdx.x & (kTX - 1);
  double cl = 1e300, arg = 1e300, dev = 0.0, bad = 0.0;
  for (int k = lane; k < kp.nxt; k += kTX) {
    const double* st = kb.strip + ((long long)par * kp.nxt + k) * 4;
    if (st[0] < cl || (st[0] == cl && st[1] < arg)) {
      cl = st[0];
      arg = st[1];
    }
    dev += st[2];
    bad = fmax(bad, st[3]);
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const double ocl = lane_xor(cl, off);
    const double oarg = lane_xor(arg, off);
    const double odev = lane_xor(dev, off);
    const double obad = lane_xor(bad, off);
    if (ocl < cl || (ocl == cl && oarg < arg)) {
      cl = ocl;
      arg = oarg;
    }
    dev += odev;
    bad = fmax(bad, obad);
  }
  if (lane == 0) {
    double* h = kb.hist + (step % kb.hist_cap) * 4;
    h[0] = double(step);
    h[1] = (kp.cl_in - cl) / kp.cl_in;        // Eq. (CL)
    h[2] = dev / (double(kp.nx) * kp.cl_in);  // Eq. (Clline)
    h[3] = arg;
    if (bad != 0.0) kb.status[0] |= 1u;       // one writing wavefront per launch
  }
}

// Block-wide sum of nv <= 4 doubles per thread of the first W wavefronts
// (fixed order: the wavefronts' values in wavefront order, then a lane
// butterfly); the result for quantity k is left in red[k][0][0]. Every thread
// of the block (NT threads) reaches every barrier. Wavefronts beyond W only
// meet the barriers; wavefronts that hold zeros leave the sum's bits as they
// are (x + 0 = x), so a block of 8 whose last 4 hold nothing sums like one of 4.
template <int W = kTY, int NT = kTX * W>
__device__ __forceinline__ void block_sum(double (*red)[W][kTX], const double* v, int nv) {
  const int tx = threadIdx.x & (kTX - 1);
  const int w = threadIdx.x / kTX;
  if (NT <= kTX * W || w < W)
    for (int k = 0; k < nv; ++k) red[k][w][tx] = v[k];
  __syncthreads();
  const int k = w;  // wavefront w sums quantity k = w (wave-uniform)
  double s = 0.0;
  if (k < nv) {
    s = red[k][0][tx];
#pragma unroll
    for (int u = 1; u < W; ++u) s += red[k][u][tx];
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) s += lane_xor(s, off);
  }
  __syncthreads();
  if (k < nv && tx == 0) red[k][0][0] = s;
  __syncthreads();
}

// One block of the fused sweep of a channel, block index b of the channel's
// own grid (lead blocks, then the tiles). jsums (with EVAL): the momentum
// column sums of level t, which steps do not carry, go to the partials of the
// other reduction slot ((t + 1) & 1, free once level t is finalized).
template <class MD, bool PULL, bool EVAL, bool SPLIT, bool NT, bool REC = false>
__device__ __forceinline__ void sweep_block(const KParams& kp, const KBufs& kb,
                                            const typename MD::St* __restrict__ src, typename MD::St* __restrict__ dst,
                                            double* __restrict__ mom, typename MD::St* __restrict__ fraw,
                                            double* __restrict__ ffull, long long t, long long t_first, int b,
                                            double (*red)[kWaves<MD>][kTX], bool jsums = false) {
  using C = typename MD::Ct;
  constexpr int W = kWaves<MD>;
  const bool px = kp.flags & LBSEP_PERIODIC_X;
  if (b < kp.lead) {
    if (b >= kp.nendb) {
      // ---- pipelined reductions of the two previous levels --------------------
      if (EVAL) return;
      const int r = b - kp.nendb;
      const int nsb = strip_blocks(kp.nxt, W);
      if (r < nsb) {
        const int bx = r * W + int(threadIdx.x / kTX);
        if (bx < kp.nxt && t - 1 >= t_first)
          strip_reduce(kp, kb, bx, t - 1, int((t - 1) & 1), kp.nrt, kb.part_stride, 2);
      } else if (r == nsb) {
        if (t - 2 >= t_first && threadIdx.x < kTX) global_reduce(kp, kb, t - 2, int((t - 2) & 1));
      }
      return;
    }
    // ---- inlet (e = 0) / outlet (e = 1) columns ------------------------------------
    // An end unit is 64 rows of one end column, held by 256 threads: lane
    // L = 4 j' + 2 s + layer holds, for row j = 64 u + j' and species s, the
    // pulled populations of the first (layer 0) or second (layer 1) inner
    // layer; layer-0 lanes also pull the boundary node itself. All these loads
    // are in flight together; Eq. (rho2) then needs the whole column's sum of
    // rho' (Eq. (rho1)) for kappa, after which the layer-0 lanes rebuild the
    // node from their own and their layer-1 neighbour's values and collide it
    // in species pairs (lanes L and L ^ 2). A block of 4 wavefronts holds one
    // unit; a block of 8 holds two: the two ends of a channel of at most 64
    // rows, else two consecutive units of one end.
    if (px) return;
    const int L = threadIdx.x & (kEndThreads - 1);
    const int h = W == 8 ? int(threadIdx.x / kEndThreads) : 0;  // half of a block of 8
    const bool both = W == 8 && kp.ny <= 64;                     // the halves are the two ends
    const bool pair_units = W == 8 && !both;                     // the halves are units u, u + 1
    auto unit_of = [&](int hh, int& ee, int& uu) {
      if (W != 8) {
        ee = b / kp.nend;
        uu = b - ee * kp.nend;
      } else if (both) {
        ee = hh;
        uu = 0;
      } else {
        const int per = kp.nendb / 2;
        ee = b / per;
        uu = 2 * (b - ee * per) + hh;
      }
    };
    int e, u;
    unit_of(h, e, u);
    const int col = e ? kp.nx - 1 : 0;
    const int l1 = e ? kp.nx - 2 : 1;
    const int l2 = e ? kp.nx - 3 : 2;  // first and second inner layers
    const int layer = L & 1;
    const int s = (L >> 1) & 1;
    const int j = u * 64 + (L >> 2);
    const bool active = j < kp.ny;
    C g[9], f[9];
    double kap = 1.0, km1 = 0.0;
#pragma unroll
    for (int i = 0; i < 9; ++i) g[i] = f[i] = C(0);
    if (PULL) {
      if (active) {
        gather1<MD, true>(kp, src, s, layer ? l2 : l1, j, t, g);
        if (layer == 0) gather1<MD, true>(kp, src, s, col, j, t, f);
      }
      // kappa needs sum_j rho'(col, j) over the whole column: thread slot L
      // adds items L, L + 256, L + 512, ... (item 4 j + 2 s + layer, 256 per
      // unit) in that order: its own unit's from the registers, the other
      // half's (units u, u + 1 of one end) through LDS, other blocks' pulled
      // again (sum only); so every block of the column forms the same sums.
      double* xch = &red[W - 1][0][0];  // 256 doubles of scratch, untouched by the block sums below
      if (pair_units) {
        if (h == 1 && active) xch[L] = double(sum9(g));
        __syncthreads();
      }
      double sums[2] = {0.0, 0.0};
      if (h == 0 || both) {
        for (int it = L; it < 4 * kp.ny; it += kEndThreads) {
          const int uk = it >> 8;  // unit of item it
          double v;
          if (uk == u) {
            v = double(sum9(g));
          } else if (pair_units && uk == u + 1) {
            v = xch[L];
          } else {
            C hv[9];
            gather1<MD, true>(kp, src, s, layer ? l2 : l1, it >> 2, t, hv);
            v = double(sum9(hv));
          }
          if (s) sums[1] += layer ? -v : 2.0 * v; else sums[0] += layer ? -v : 2.0 * v;
        }
      }
      // the two ends of a block of 8 sum apart (quantities 2 e + s); a zero
      // added to a sum leaves its bits, so each end's sums are those of a
      // block of 4 that holds the unit alone
      const double q4[4] = {both && h ? 0.0 : sums[0], both && h ? 0.0 : sums[1], both && h ? sums[0] : 0.0,
                            both && h ? sums[1] : 0.0};
      block_sum<W>(red, q4, both ? 4 : 2);
      const double n = double(kp.ny), sum = red[(both ? 2 * h : 0) + s][0][0];
      __syncthreads();  // red is reused by the block sum below
      if (MD::kDev) {
        // sum_j rho' = n rho0(col) + sum (deviation sums)
        const double r0 = ref_rho(kp, s, col);
        km1 = (n * (kp.rho_bc[e][s] - r0) - sum) / (n * r0 + sum);
        kap = 1.0 + km1;
      } else {
        kap = n * kp.rho_bc[e][s] / sum;
        km1 = kap - 1.0;
      }
      // layer-1 values to the layer-0 lane of the same (row, species)
      C g2[9];
#pragma unroll
      for (int i = 0; i < 9; ++i) g2[i] = lane_xor(g[i], 1);
      if (active && layer == 0) end_rebuild<MD>(kp, e, s, col, kap, km1, g, g2, f);
    } else {
      if (active && layer == 0) gather1<MD, false>(kp, src, s, col, j, t, f);
    }
    double acc2[2] = {0.0, 0.0};
    process_pair<MD, EVAL, 2, true, false, REC>(kp, col, j, t, s, active && layer == 0, f, dst, mom, fraw, ffull, acc2,
                                                reinterpret_cast<double*>(fraw));
    if (EVAL && !jsums) return;
    // the unit sums: quantity 4 h + q of half h (q: n_a, n_b, rho_a u_ax, rho_b u_bx)
    double a8[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    const double acc[4] = {s ? 0.0 : acc2[0], s ? acc2[0] : 0.0, s ? 0.0 : acc2[1], s ? acc2[1] : 0.0};
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if (h == 0) a8[q] = acc[q];
      else a8[4 + q] = acc[q];
    }
    constexpr int kUnitSums = W == 8 ? 8 : 4;
    block_sum<W>(red, a8, kUnitSums);
    // a step: all four sums of level t; an evaluation sweep: the momenta, to the other slot
    const int tq = threadIdx.x;
    if (tq < kUnitSums && (!EVAL || (tq & 3) >= 2)) {
      int ee, uu;
      unit_of(tq >> 2, ee, uu);
      if (uu * 64 < kp.ny)
        kb.endsum[((((EVAL ? t + 1 : t) & 1) * 2 + ee) * kMaxEnd + uu) * 4 + (tq & 3)] = red[tq][0][0];
    }
    return;
  }
  // ---- interior tile --------------------------------------------------------------
  // tiles in grid order, without regard to XCDs: the blocks in flight on all
  // XCDs then read and write one compact stretch of the state (measured on
  // 512 x 10240 FP32: 5% faster than giving each XCD a contiguous share)
  const int lin = b - kp.lead;
  if (lin >= kp.tiles) return;
  // row bands (one lane per node) or column strips (lane pairs)
  int bx, by;
  if (kp.flags & kRowMajorTiles) {
    by = lin / kp.ntx;
    bx = lin - by * kp.ntx;
  } else {
    bx = lin / kp.nrt;
    by = lin - bx * kp.nrt;
  }
  const int lane = threadIdx.x & (kTX - 1);
  // the wave's row within the tile, uniform across the wave: row bases of the
  // state buffers then stay in scalar registers
  const int ty = __builtin_amdgcn_readfirstlane(threadIdx.x / kTX);
  if (SPLIT) {
    // 32 columns x (W rpt) rows; lanes 0-31 hold species a, 32-63 species b
    const int s = lane >> 5;
    const int cx = lane & 31;
    const int x = bx * 32 + cx;
    const bool xin = (x < kp.nx) && (px || (x > 0 && x < kp.nx - 1));
    double acc[2] = {0.0, 0.0};
#pragma unroll 1
    for (int r = 0; r < kp.rpt; ++r) {
      const int j = by * (W * kp.rpt) + r * W + ty;
      if (j < kp.ny) {  // wave-uniform
        C f[9];
        if (xin) gather1<MD, PULL>(kp, src, s, x, j, t, f);
        process_pair<MD, EVAL, 32, true, false, REC>(kp, x, j, t, s, xin, f, dst, mom, fraw, ffull, acc,
                                                     reinterpret_cast<double*>(fraw));
      }
    }
    if (EVAL && !jsums) return;
    // per-column sums of this row tile: quantity q = s (n_s) and 2 + s
    // (rho_s u_sx); the densities in a step, the momenta in an evaluation sweep
    red[s][ty][cx] = acc[0];
    red[2 + s][ty][cx] = acc[1];
    __syncthreads();
    if (threadIdx.x < 64) {
      const int q = (threadIdx.x >> 5) + (EVAL ? 2 : 0), c = threadIdx.x & 31;
      const int xc = bx * 32 + c;
      if (xc < kp.nx) {
        double v = red[q][0][c];
#pragma unroll
        for (int u = 1; u < W; ++u) v += red[q][u][c];
        kb.partials[((EVAL ? t + 1 : t) & 1) * kb.part_stride + ((long long)q * kp.nrt + by) * kp.pitch + xc] = v;
      }
    }
  } else {
    // 64 columns x (W rpt) rows, one lane per node
    const int x = bx * kTX + lane;
    const bool xin = (x < kp.nx) && (px || (x > 0 && x < kp.nx - 1));
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 1
    for (int r = 0; r < kp.rpt; ++r) {
      const int j = by * (W * kp.rpt) + r * W + ty;
      if (xin && j < kp.ny) {
        C fa[9], fb[9];
        gather_pair<MD, PULL>(kp, src, x, j, t, fa, fb);
        process_node<MD, EVAL, NT, REC>(kp, x, j, t, fa, fb, dst, mom, fraw, ffull, acc,
                                        reinterpret_cast<double*>(fraw));
      }
    }
    if (EVAL && !jsums) return;
    // per-column sums of this row tile (W wavefronts -> 1), quantity q = ty
    // (wavefronts 0-3): the densities in a step, the momenta in an evaluation
    // sweep
#pragma unroll
    for (int q = 0; q < 4; ++q) red[q][ty][lane] = acc[q];
    __syncthreads();
    if (x < kp.nx && ty < 4 && (ty >= 2) == EVAL) {
      double v = red[ty][0][lane];
#pragma unroll
      for (int u = 1; u < W; ++u) v += red[ty][u][lane];
      kb.partials[((EVAL ? t + 1 : t) & 1) * kb.part_stride + ((long long)ty * kp.nrt + by) * kp.pitch + x] = v;
    }
  }
}

// One-level tiles are dealt out in groups of 8 kXcdRun: the hardware hands
// block k of a launch to XCD k mod 8, so placing tile kXcdRun j + t of a group
// at slot j + 8 t gives each XCD kXcdRun consecutive tiles (x-neighbours in a
// row band, y-neighbours in a column strip) back to back; the halo lines they
// share then come from the XCD's own L2 instead of the memory side (64-member
// table, FP32: fetched plus written bytes 1.109 -> 1.050 times the
// algorithmic ones). A last partial group keeps the plain order. k_sweep maps
// its block index here; batches order their block table the same way on the
// host.
constexpr int kXcdRun = 4;

__device__ __forceinline__ int xcd_run_block(const KParams& kp, int b) {
  constexpr int grp = 8 * kXcdRun;
  const int lin = b - kp.lead;
  if (lin < 0 || lin >= kp.tiles / grp * grp) return b;
  const int s = lin % grp;
  return kp.lead + (lin - s) + kXcdRun * (s % 8) + s / 8;
}

// REC (a recording step of an FP64 channel): besides the step, ffull receives
// the pulled (pre-collision) populations and fraw the post-collision ones,
// both dense [2][9][ny][nx].
template <class MD, bool PULL, bool EVAL, bool SPLIT, bool NT, bool REC = false>
__global__ __launch_bounds__(kTX * kWaves<MD>) void k_sweep(KParams kp, KBufs kb, const typename MD::St* __restrict__ src,
                                                    typename MD::St* __restrict__ dst, double* __restrict__ mom,
                                                    typename MD::St* __restrict__ fraw,
                                                    double* __restrict__ ffull, long long t,
                                                    long long t_first, int jsums) {
  __shared__ double red[kWaves<MD>][kWaves<MD>][kTX];  // up to W quantities (inlet/outlet unit sums)
  sweep_block<MD, PULL, EVAL, SPLIT, NT, REC>(kp, kb, src, dst, mom, fraw, ffull, t, t_first,
                                              xcd_run_block(kp, (int)blockIdx.x), red, jsums != 0);
}

// A batch of channels swept by one launch: entry i holds channel i's constants,
// reduction buffers and state buffers. Block k of the batch grid runs block
// blk_ref[k].y of the launch of channel blk_ref[k].x alone; the grid lists
// every member's end blocks first, then every member's reduction blocks, then
// the members' tiles: the end blocks, the longest, start first rather than
// stretching the end of the launch.
struct BatchEntry {
  KParams kp;
  KBufs kb;
  void* f[2];          // the channel's two state buffers
  long long t0;        // channel level when the batch's step counter was 0
  long long t_first;   // first level with a history record
  int cur0;            // buffer holding the post-collision state at counter 0
  int split;           // tile kind: lane pair per node (1) or one lane per node (0)
  int pad;
};

// Batch step k = *counter + k_local: every channel advances by one level.
template <class MD, bool NT>
__global__ __launch_bounds__(kTX * kWaves<MD>) void k_sweep_batch(const BatchEntry* __restrict__ tab,
                                                          const int2* __restrict__ blk_ref,
                                                          const long long* __restrict__ counter, int k_local) {
  __shared__ double red[kWaves<MD>][kWaves<MD>][kTX];  // up to W quantities (inlet/outlet unit sums)
  using S = typename MD::St;
  const int2 ref = blk_ref[blockIdx.x];
  const BatchEntry& e = tab[ref.x];
  const long long k = *counter + k_local;
  const int c = (e.cur0 + (int)(k & 1)) & 1;
  const S* src = static_cast<const S*>(e.f[c]);
  S* dst = static_cast<S*>(e.f[c ^ 1]);
  const int b = ref.y;
  if (e.split)
    sweep_block<MD, true, false, true, false>(e.kp, e.kb, src, dst, nullptr, nullptr, nullptr, e.t0 + k + 1,
                                              e.t_first, b, red);
  else
    sweep_block<MD, true, false, false, NT>(e.kp, e.kb, src, dst, nullptr, nullptr, nullptr, e.t0 + k + 1,
                                            e.t_first, b, red);
}

__global__ void k_batch_advance(long long* counter, long long n) {
  if (blockIdx.x == 0 && threadIdx.x == 0) *counter += n;
}

// Completes the records of levels t - 1 and t (reads after the last sweep):
// phase 0 reduces the strips of level t (blocks 0 .. nxt-1) and finishes level
// t - 1 (block nxt); phase 1 finishes level t.
// ---- two time levels per launch ---------------------------------------------
// k_sweep2 advances the state by nlev = 1 or 2 levels in one launch, on a
// channel of at most 64 rows. A tile of kW2 wavefronts x 64 lanes computes the
// first level on its rows and columns plus a one-node halo (wavefront w: row
// 6 by - 1 + w; lane l: column 2 + 62 bx + l), keeps those post-collision
// pairs in LDS in the storage type (the values the next pull would read back
// from memory), and computes the second level on the 6 x 62 nodes it owns
// from LDS alone. The inlet and outlet columns couple every row through kappa
// (Eq. (rho2)): one block per end computes the first level on its four
// outermost columns for all rows (in LDS), takes kappa of the second level
// from there, and computes the second level of its three outermost columns.
// The tiles own the columns between, so that none of them needs kappa. kappa
// is summed in the order of the single-level end blocks, so every node goes
// through the same arithmetic as in two single-level sweeps: the states are
// bitwise those. The lead blocks reduce the row-tile partials of earlier
// levels (level lists from the host, four slots by level mod 4).
constexpr int kW2 = 8;            // wavefronts per block
constexpr int kT2 = kW2 * kTX;    // threads per block
constexpr int kR2 = kW2 - 2;      // rows a tile owns
constexpr int kC2 = kTX - 2;      // columns a tile owns

// Tiling and levels of one k_sweep2 launch (its own argument, so that the
// single-level kernels keep their argument block as small as it was).
struct Lv2 {
  int ntx, nrt;            // 62-column tile strips, 6-row tiles
  int tiles, chunk;        // ntx * nrt, ceil(tiles / 8)
  int lead;                // lead blocks (multiple of 8) before the first tile
  long long part_stride;   // elements of one partials slot: 4 * nrt * pitch
  long long t1;            // first level this launch computes (current level + 1)
  int nlev;                // levels computed: 1 or 2
  int reduce;              // write row-tile partials and end sums (0: a replay)
  long long strip[2];      // levels to strip-reduce, -1 = none
  long long glob[2];       // levels to reduce to a record, -1 = none
};

// kappa of Eq. (rho2) for end e from each thread's two column sums
// (species 0, 1) of rho' (Eq. (rho1)): block_sum, then kap[s] = kappa and
// km1[s] = kappa - 1 for both species, in every thread. Every thread of the
// block must call it (barriers).
template <class MD>
__device__ __forceinline__ void kappa_from_sums(const KParams& kp, int e, double (*red)[kTY][kTX], double sums[2],
                                                double kap[2], double km1[2]) {
  const int col = e ? kp.nx - 1 : 0;
  block_sum<kTY, kT2>(red, sums, 2);
  const double n = double(kp.ny);
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    const double sum = red[s][0][0];
    // a select, not an index by e: e may be a runtime value here, and a
    // dynamic index would move this kernel's parameter block to scratch memory
    const double rbc = e ? kp.rho_bc[1][s] : kp.rho_bc[0][s];
    if (MD::kDev) {
      // sum_j rho' = n rho0(col) + sum (deviation sums)
      const double r0 = ref_rho(kp, s, col);
      km1[s] = (n * (rbc - r0) - sum) / (n * r0 + sum);
      kap[s] = 1.0 + km1[s];
    } else {
      kap[s] = n * rbc / sum;
      km1[s] = kap[s] - 1.0;
    }
  }
  __syncthreads();  // red is reused by the caller
}

// kappa of end e from the values v[it] = rho of the pulled populations of the
// two inner layers, it = 4 row + 2 species + layer, in LDS, summed in the
// order of the single-level end blocks: thread L < 256 adds item L and then,
// for more than 64 rows, item L + 256 (the single-level end blocks of rows
// 0-63 and 64-127 both hold that pair in thread L), then kappa_from_sums.
// Every thread of the block must call it (barriers).
template <class MD>
__device__ __forceinline__ void kappa_from_values(const KParams& kp, int e, const double* v, double (*red)[kTY][kTX],
                                                  double kap[2], double km1[2]) {
  double sums[2] = {0.0, 0.0};
  const int it = threadIdx.x;
  if (it < kEndThreads) {
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const int item = it + k * kEndThreads;
      if (item < 4 * kp.ny) {
        const int ss = (item >> 1) & 1, ll = item & 1;
        if (ss)
          sums[1] += ll ? -v[item] : 2.0 * v[item];
        else
          sums[0] += ll ? -v[item] : 2.0 * v[item];
      }
    }
  }
  kappa_from_sums<MD>(kp, e, red, sums, kap, km1);
}

// The pulled populations of node (lane l, wavefront w, row j) of a tile from
// the first level's post-collision pairs in LDS: gather_pair with LDS as the
// source (same deviation correction, same DBB).
template <class MD>
__device__ __forceinline__ void lds_gather(const KParams& kp, const typename MD::Pt (*lds)[9][kTX], int l, int w,
                                           int x, int j, long long t, typename MD::Ct fa[9], typename MD::Ct fb[9]) {
  using C = typename MD::Ct;
  const bool bot = j == 0, top = j == kp.ny - 1;
  const int wm = bot ? w : w - 1, wp = top ? w : w + 1;  // the wall-crossing loads are discarded
  const int sl[9] = {l, l - 1, l, l + 1, l, l - 1, l + 1, l + 1, l - 1};
  const int sw[9] = {w, w, wm, w, wp, wm, wm, wp, wp};
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    const typename MD::Pt v = lds[sw[i]][i][sl[i]];
    fa[i] = C(v[0]);
    fb[i] = C(v[1]);
  }
  if constexpr (MD::kDev) {
    add_stream_corr<MD>(kp, x, j, t, 0, fa);
    add_stream_corr<MD>(kp, x, j, t, 1, fb);
  }
  if (bot || top) {
    const int o0 = bot ? 4 : 2, o1 = bot ? 7 : 5, o2 = bot ? 8 : 6;
    dbb_pair<MD>(kp, bot, lds[w][o0][l], lds[w][o1][l], lds[w][o2][l], fa, fb);
  }
}

// Sum over the kW2 wavefronts of quantity q per lane, first four quantities
// (red[q][w][lane] written by every wavefront beforehand; fixed order).
__device__ __forceinline__ double wave_column_sum(const double (*red)[kW2][kTX], int q, int lane, int w0, int w1) {
  double v = 0.0;
  for (int w = w0; w <= w1; ++w) v += red[q][w][lane];
  return v;
}

// The end strip of a two-level launch in LDS: column c (0 = the end column,
// counted inwards), row j, direction i; at most 128 rows in the deviation
// modes (one node per thread of the 512-thread block), 64 in FP64 (a lane
// pair per node, and twice the bytes per population). The two-level kernels
// are instantiated per strip size: MD there is StripMode<mode, R>, R = 64 for
// channels of at most 64 rows (the smaller LDS strips and end-column sums
// keep those channels as fast as before the 128-row strips: 64x1280 FP32
// 6.25 -> 5.86 us per level) and 128 above.
template <class MD, int R>
struct StripMode : MD {
  static constexpr int kStripRows = R;
};
template <class MD>
constexpr int kStripRowsOf = MD::kStripRows;
constexpr int strip_max_rows(int dtype) { return dtype == LBSEP_F64 ? 64 : 128; }

// Pulled populations of node (c, j) of end e's strip from its post-collision
// pairs Q (storage type): gather_pair with the strip as the source.
template <class MD>
__device__ __forceinline__ void strip_gather(const KParams& kp, const typename MD::Pt (*Q)[kStripRowsOf<MD>][9], int e,
                                             int c, int j, long long t, typename MD::Ct fa[9], typename MD::Ct fb[9]) {
  using C = typename MD::Ct;
  const bool bot = j == 0, top = j == kp.ny - 1;
  const int jm = bot ? j : j - 1, jp = top ? j : j + 1;  // the wall-crossing loads are discarded
  // strip columns of x - 1 and x + 1 (kept in range at the end column, as gather_pair does)
  const int cm = max(e ? c + 1 : c - 1, 0), cp = max(e ? c - 1 : c + 1, 0);
  const int sc[9] = {c, cm, c, cp, c, cm, cp, cp, cm};
  const int sy[9] = {j, j, jm, j, jp, jm, jm, jp, jp};
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    const typename MD::Pt v = Q[sc[i]][sy[i]][i];
    fa[i] = C(v[0]);
    fb[i] = C(v[1]);
  }
  if constexpr (MD::kDev) {
    const int x = e ? kp.nx - 1 - c : c;
    add_stream_corr<MD>(kp, x, j, t, 0, fa);
    add_stream_corr<MD>(kp, x, j, t, 1, fb);
  }
  if (bot || top) {
    const int o0 = bot ? 4 : 2, o1 = bot ? 7 : 5, o2 = bot ? 8 : 6;
    dbb_pair<MD>(kp, bot, Q[c][j][o0], Q[c][j][o1], Q[c][j][o2], fa, fb);
  }
}

// Columns of each end a two-level launch gives to its end block: the end
// column and the next two (counted inwards). The tiles own the columns
// between, so that no tile touches an end column or needs kappa.
constexpr int kEndCols = 3;

// Per-node sums of one level of an end block, by column, quantity (n_a, n_b,
// rho_a u_ax, rho_b u_bx) and row, in LDS while the block reduces them.
template <class MD>
using EndSums = double[kEndCols][4][kStripRowsOf<MD>];

// A thread's own sums of the nodes it computed, per level: column c, row j,
// the quantities q (all four, or with a lane pair per node q = s and 2 + s).
struct EndNodeSums {
  double v[2][4];
  int c[2], j[2], s[2];  // s = -1: all four quantities
  bool on[2];
};

// End block of a two-level launch, one lane per node: task (c, j) = (thread
// % 4, thread / 4), so a quad holds the four outermost columns of row j; the
// first level of those columns stays in LDS. Phase 1 pulls every node once:
// the two inner layers' values give kappa (kappa_from_values) and, moved to
// the end column's lane within the quad, its rebuild; the four columns
// collide into LDS in the storage type (nlev = 1: columns 0 to 2 are stored to
// dst instead). Phase 2 pulls columns 0 to 2 from LDS, takes the second kappa
// the same way, rebuilds the end column and collides and stores the three
// columns. ns: the node's sums per level.
template <class MD, bool NT>
__device__ __forceinline__ void end_block2_node(const KParams& kp, const typename MD::St* __restrict__ src,
                                                typename MD::St* __restrict__ dst, int e, int nlev, long long t1,
                                                typename MD::Pt (*Q)[kStripRowsOf<MD>][9], double* Kv,
                                                double (*redk)[kTY][kTX], EndNodeSums& ns) {
  using C = typename MD::Ct;
  const int sgn = e ? -1 : 1, col = e ? kp.nx - 1 : 0;
  const int c = threadIdx.x & 3, j = threadIdx.x >> 2;
  const bool act = j < kp.ny;  // uniform over a quad
  const int x = col + sgn * c;
  double kap[2], km1[2];
  double sums1[4] = {0.0, 0.0, 0.0, 0.0}, sums2[4] = {0.0, 0.0, 0.0, 0.0};
  // the end column's rebuild from the first and second inner layers' pulled
  // populations, lanes c = 1 and 2 of the same quad (exact moves)
  auto rebuild = [&](C fa[9], C fb[9]) {
    C g1[9], g2[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      g1[i] = lane_xor(fa[i], 1);
      g2[i] = lane_xor(fa[i], 2);
    }
    if (c == 0) end_rebuild<MD>(kp, e, 0, col, kap[0], km1[0], g1, g2, fa);
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      g1[i] = lane_xor(fb[i], 1);
      g2[i] = lane_xor(fb[i], 2);
    }
    if (c == 0) end_rebuild<MD>(kp, e, 1, col, kap[1], km1[1], g1, g2, fb);
  };
  // ---- first level
  C fa[9], fb[9];
  if (act) gather_pair<MD, true>(kp, src, x, j, t1, fa, fb);
  if (act && (c == 1 || c == 2)) {
    Kv[4 * j + (c - 1)] = double(sum9(fa));
    Kv[4 * j + 2 + (c - 1)] = double(sum9(fb));
  }
  __syncthreads();
  kappa_from_values<MD>(kp, e, Kv, redk, kap, km1);
  if (act) {
    rebuild(fa, fb);
    const NodeState<C> st = node_moments<MD, false>(kp, x, j, fa, fb, nullptr, nullptr, nullptr, sums1);
    node_collide_only<MD>(kp, x, j, t1, fa, fb, st);
    if (nlev == 2) {
#pragma unroll
      for (int i = 0; i < 9; ++i) {
        typename MD::Pt v;
        v[0] = typename MD::St(fa[i]);
        v[1] = typename MD::St(fb[i]);
        Q[c][j][i] = v;
      }
    } else if (c < kEndCols) {
      node_store<MD, NT>(kp, x, j, fa, fb, dst);
    }
  }
  if (nlev == 2) {
    __syncthreads();
    // ---- second level: columns 0 to 2 (lanes c = 3 idle)
    if (act && c < kEndCols) {
      strip_gather<MD>(kp, Q, e, c, j, t1 + 1, fa, fb);
      if (c > 0) {
        Kv[4 * j + (c - 1)] = double(sum9(fa));
        Kv[4 * j + 2 + (c - 1)] = double(sum9(fb));
      }
    }
    __syncthreads();
    kappa_from_values<MD>(kp, e, Kv, redk, kap, km1);
    if (act && c < kEndCols) {
      rebuild(fa, fb);
      const NodeState<C> st = node_moments<MD, false>(kp, x, j, fa, fb, nullptr, nullptr, nullptr, sums2);
      node_collide_only<MD>(kp, x, j, t1 + 1, fa, fb, st);
      node_store<MD, NT>(kp, x, j, fa, fb, dst);
    }
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    ns.v[0][q] = sums1[q];
    ns.v[1][q] = sums2[q];
  }
#pragma unroll
  for (int l = 0; l < 2; ++l) {
    ns.c[l] = c;
    ns.j[l] = j;
    ns.s[l] = -1;
    ns.on[l] = act && c < kEndCols && l < nlev;
  }
}

// end_rebuild of species s (a runtime value) at the end column from the inner
// layers' pulled populations P[layer][j][i][species] in LDS; one branch per
// species keeps the parameter indexes constant.
template <class MD>
__device__ __forceinline__ void strip_rebuild1(const KParams& kp, int e, int col, int j, int s,
                                               const typename MD::Ct (*P)[kStripRowsOf<MD>][9][2], const double kap[2],
                                               const double km1[2], typename MD::Ct f[9]) {
  using C = typename MD::Ct;
  C g1[9], g2[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    g1[i] = P[0][j][i][s];
    g2[i] = P[1][j][i][s];
  }
  if (s)
    end_rebuild<MD>(kp, e, 1, col, kap[1], km1[1], g1, g2, f);
  else
    end_rebuild<MD>(kp, e, 0, col, kap[0], km1[0], g1, g2, f);
}

// The same with a lane pair per node: thread t takes species s = t % 2 of a
// node, the two species of a node sit in adjacent lanes and collide as a lane
// pair (process_pair: the same arithmetic as one lane per node, half the chain
// per lane). Phase 1: node (column c = (t / 2) % 4 from the end, row
// j = t / 8); phase 2: column c = t / 128, row j = (t / 2) % 64.
template <class MD, bool NT>
__device__ __forceinline__ void end_block2_pair(const KParams& kp, const typename MD::St* __restrict__ src,
                                                typename MD::St* __restrict__ dst, int e, int nlev, long long t1,
                                                typename MD::Pt (*Q)[kStripRowsOf<MD>][9],
                                                typename MD::Ct (*P)[kStripRowsOf<MD>][9][2], double* Kv,
                                                double (*redk)[kTY][kTX], EndNodeSums& ns) {
  using C = typename MD::Ct;
  using S = typename MD::St;
  const int sgn = e ? -1 : 1, col = e ? kp.nx - 1 : 0;
  const int s = threadIdx.x & 1, c = (threadIdx.x >> 1) & 3, j = threadIdx.x >> 3;
  const bool act = j < kp.ny;
  const int x = col + sgn * c;
  double kap[2], km1[2];
  double sums1[2] = {0.0, 0.0}, sums2[2] = {0.0, 0.0};
  C f[9];
  // ---- first level
  {
    C fa[9], fb[9];
    if (act) gather_pair<MD, true>(kp, src, x, j, t1, fa, fb);
#pragma unroll
    for (int i = 0; i < 9; ++i) f[i] = s ? fb[i] : fa[i];
  }
  if (act && (c == 1 || c == 2)) {
#pragma unroll
    for (int i = 0; i < 9; ++i) P[c - 1][j][i][s] = f[i];
    Kv[4 * j + 2 * s + (c - 1)] = double(sum9(f));
  }
  __syncthreads();
  kappa_from_values<MD>(kp, e, Kv, redk, kap, km1);
  if (act && c == 0) strip_rebuild1<MD>(kp, e, col, j, s, P, kap, km1, f);
  process_pair<MD, false, 1, false, true>(kp, x, j, t1, s, act, f, nullptr, nullptr, nullptr, nullptr, sums1);
  if (nlev == 2) {
    if (act)
#pragma unroll
      for (int i = 0; i < 9; ++i) reinterpret_cast<S*>(&Q[c][j][i])[s] = S(f[i]);
  } else if (act && c < kEndCols) {
#pragma unroll
    for (int i = 0; i < 9; ++i) *pop_at(kp, dst, s, i, j, x) = S(f[i]);
  }
  const int c2 = threadIdx.x >> 7, j2 = (threadIdx.x >> 1) & 63;
  const bool act2 = j2 < kp.ny && c2 < kEndCols;
  if (nlev == 2) {
    __syncthreads();
    // ---- second level: columns 0 to 2
    if (act2) {
      C fa[9], fb[9];
      strip_gather<MD>(kp, Q, e, c2, j2, t1 + 1, fa, fb);
#pragma unroll
      for (int i = 0; i < 9; ++i) f[i] = s ? fb[i] : fa[i];
      if (c2 > 0) {
#pragma unroll
        for (int i = 0; i < 9; ++i) P[c2 - 1][j2][i][s] = f[i];
        Kv[4 * j2 + 2 * s + (c2 - 1)] = double(sum9(f));
      }
    }
    __syncthreads();
    kappa_from_values<MD>(kp, e, Kv, redk, kap, km1);
    if (c2 < kEndCols) {  // both lanes of each pair (wavefronts 0 to 5)
      if (act2 && c2 == 0) strip_rebuild1<MD>(kp, e, col, j2, s, P, kap, km1, f);
      process_pair<MD, false, 1, true, true>(kp, col + sgn * c2, j2, t1 + 1, s, act2, f, dst, nullptr, nullptr, nullptr,
                                             sums2);
    }
  }
  ns.v[0][s] = sums1[0];
  ns.v[0][2 + s] = sums1[1];
  ns.v[1][s] = sums2[0];
  ns.v[1][2 + s] = sums2[1];
  ns.c[0] = c;
  ns.j[0] = j;
  ns.c[1] = c2;
  ns.j[1] = j2;
  ns.s[0] = ns.s[1] = s;
  ns.on[0] = act && c < kEndCols;
  ns.on[1] = nlev == 2 && act2;
}

// Lane pairs in the two-level end blocks: in FP64 the wall functions dominate a
// node's chain and splitting them over the pair shortens the inlet/outlet path
// (measured on 64 x 1280); in the deviation modes the pair's swaps cost more
// than they save.
template <class MD>
constexpr bool kPairEnd = !MD::kDev;

// Inlet (e = 0) or outlet (e = 1) block of k_sweep2 (a channel of at most
// 128 rows, 64 in FP64): columns 0 to 2 from the end at every level the
// launch computes, then their sums over the rows, level by level: the end
// column's to the end sums (end block 0 of the level's slot, zeros to the
// rest), the other two columns' to row tile 0 of the partials (zeros to the
// other row tiles). The zeros go out first (no reduction of this launch reads
// these levels' slots); each sum is a fixed two-stage order (an eighth of the
// strip's rows per thread, then the eight partial sums).
template <class MD, bool NT>
__device__ __forceinline__ void end_block2(const KParams& kp, const KBufs& kb, const Lv2& lv,
                                           const typename MD::St* __restrict__ src, typename MD::St* __restrict__ dst,
                                           int e, double (*red)[kW2][kTX], double (*redk)[kTY][kTX],
                                           typename MD::Pt (*Q)[kStripRowsOf<MD>][9],
                                           typename MD::Ct (*P)[kStripRowsOf<MD>][9][2], double* Kv) {
  if (lv.nlev == 0) return;  // a reductions-only launch
  constexpr int kRows = kStripRowsOf<MD>;
  static_assert(sizeof(EndSums<MD>) <= sizeof(double) * 4 * kW2 * kTX, "one level's end sums fit the reduction scratch");
  const int sgn = e ? -1 : 1, col = e ? kp.nx - 1 : 0;
  const int t = threadIdx.x;
  if (lv.reduce) {
    const int nzp = 2 * 4 * (lv.nrt - 1), nze = 4 * (kp.nend - 1);  // per level
    for (int z = t; z < lv.nlev * (nzp + nze); z += kT2) {
      const int lev = z / (nzp + nze), r = z - lev * (nzp + nze);
      const long long level = lv.t1 + lev;
      if (r < nzp) {  // column 1 + r / (4 (nrt - 1)), quantity, row tile >= 1
        const int c = 1 + r / (4 * (lv.nrt - 1)), q = (r / (lv.nrt - 1)) % 4, by = 1 + r % (lv.nrt - 1);
        kb.partials[(level & 3) * lv.part_stride + ((long long)q * lv.nrt + by) * kp.pitch + col + sgn * c] = 0.0;
      } else {  // end block >= 1
        const int q = (r - nzp) % 4, blk = 1 + (r - nzp) / 4;
        kb.endsum[(((level & 3) * 2 + e) * kMaxEnd + blk) * 4 + q] = 0.0;
      }
    }
  }
  EndNodeSums ns;
  if constexpr (kPairEnd<MD>)
    end_block2_pair<MD, NT>(kp, src, dst, e, lv.nlev, lv.t1, Q, P, Kv, redk, ns);
  else
    end_block2_node<MD, NT>(kp, src, dst, e, lv.nlev, lv.t1, Q, Kv, redk, ns);
  if (!lv.reduce) return;  // uniform over the block
  // per level: the nodes' sums into LDS by (column, quantity, row), then sum
  // k = (column, quantity): thread G k + g adds rows 8 g .. 8 g + 7 (G =
  // kRows / 8 groups) into Kv (free once kappa is taken), then thread k adds
  // the G group sums in order (groups beyond the channel's rows hold zeros,
  // so both strip sizes give a channel of at most 64 rows the same sums)
  EndSums<MD>& V = *reinterpret_cast<EndSums<MD>*>(&red[0][0][0]);
  constexpr int kGroups = kRows / 8;
  constexpr int nsum = kEndCols * 4;
  static_assert(kGroups * nsum <= 4 * kRows, "the partial sums fit Kv");
#pragma unroll
  for (int lev = 0; lev < 2; ++lev) {
    if (lev >= lv.nlev) break;  // uniform over the block
    __syncthreads();  // red and Kv are free (the last kappa, or the previous level's sums, are read)
    if (ns.on[lev])
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (ns.s[lev] < 0 || q == ns.s[lev] || q == 2 + ns.s[lev]) V[ns.c[lev]][q][ns.j[lev]] = ns.v[lev][q];
    __syncthreads();
    if (t < kGroups * nsum) {
      const int k = t / kGroups, g = t - k * kGroups;
      const double* v = V[k / 4][k % 4];
      double a = 0.0;
#pragma unroll
      for (int r = 0; r < 8; ++r)
        if (8 * g + r < kp.ny) a += v[8 * g + r];
      Kv[t] = a;
    }
    __syncthreads();
    if (t < nsum) {
      double a = 0.0;
#pragma unroll
      for (int g = 0; g < kGroups; ++g) a += Kv[kGroups * t + g];
      const int c = t / 4, q = t % 4;
      const long long level = lv.t1 + lev;
      if (c == 0)
        kb.endsum[(((level & 3) * 2 + e) * kMaxEnd) * 4 + q] = a;
      else
        kb.partials[(level & 3) * lv.part_stride + (long long)q * lv.nrt * kp.pitch + col + sgn * c] = a;
    }
  }
}

// Tile of k_sweep2 (see above): owns columns 3 .. nx - 4 of its rows; its
// halo columns (2 and nx - 3 at the ends) are ordinary interior nodes, so no
// tile needs kappa. Lanes beyond the owned range compute values no owned node
// reads.
template <class MD, bool NT>
__device__ __forceinline__ void tile2(const KParams& kp, const KBufs& kb, const Lv2& lv,
                                      const typename MD::St* __restrict__ src, typename MD::St* __restrict__ dst,
                                      int b, typename MD::Pt (*lds)[9][kTX], double (*red)[kW2][kTX]) {
  using C = typename MD::Ct;
  const int xcd = b & 7;
  const int k = (b - lv.lead) >> 3;
  const int lin = xcd * lv.chunk + k;
  if (lin >= lv.tiles) return;  // uniform over the block
  // column strips in order: an XCD's tiles share their halo rows in its L2, and
  // the first and last strips sit on the XCDs of the inlet and outlet blocks
  const int bx = lin / lv.nrt, by = lin - bx * lv.nrt;
  const int lane = threadIdx.x & (kTX - 1);
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kTX);
  const int x0 = kEndCols + kC2 * bx;  // first owned column
  const int x = x0 - 1 + lane;
  const int j = by * kR2 - 1 + w;
  const bool in_j = j >= 0 && j < kp.ny;
  const bool valid = x < kp.nx && in_j;
  const bool own_x = lane >= 1 && lane <= kC2 && x <= kp.nx - 1 - kEndCols;
  const bool own = own_x && w >= 1 && w <= kR2 && j < kp.ny;
  // ---- first level: own nodes and halo
  C fa[9], fb[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) fa[i] = fb[i] = C(0);
  if (valid) gather_pair<MD, true>(kp, src, x, j, lv.t1, fa, fb);
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  if (valid) {
    double tmp[4] = {0.0, 0.0, 0.0, 0.0};
    const NodeState<C> st = node_moments<MD, false>(kp, x, j, fa, fb, nullptr, nullptr, nullptr, tmp);
    if (own)
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[q] = tmp[q];
    node_collide_only<MD>(kp, x, j, lv.t1, fa, fb, st);
  }
  if (lv.nlev == 2) {
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      typename MD::Pt v;
      v[0] = typename MD::St(fa[i]);
      v[1] = typename MD::St(fb[i]);
      lds[w][i][lane] = v;
    }
  } else if (own) {
    node_store<MD, NT>(kp, x, j, fa, fb, dst);
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) red[q][w][lane] = acc[q];
  __syncthreads();
  if (lv.reduce && w < 4 && own_x) {
    const long long level = lv.t1;
    kb.partials[(level & 3) * lv.part_stride + ((long long)w * lv.nrt + by) * kp.pitch + x] =
        wave_column_sum(red, w, lane, 1, kR2);
  }
  if (lv.nlev == 1) return;  // uniform over the block
  // ---- second level: own nodes from LDS
#pragma unroll
  for (int q = 0; q < 4; ++q) acc[q] = 0.0;
  if (own) {
    C ha[9], hb[9];
    lds_gather<MD>(kp, lds, lane, w, x, j, lv.t1 + 1, ha, hb);
    double tmp[4] = {0.0, 0.0, 0.0, 0.0};
    const NodeState<C> st = node_moments<MD, false>(kp, x, j, ha, hb, nullptr, nullptr, nullptr, tmp);
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[q] = tmp[q];
    node_collide_only<MD>(kp, x, j, lv.t1 + 1, ha, hb, st);
    node_store<MD, NT>(kp, x, j, ha, hb, dst);
  }
  __syncthreads();  // the first level's sums are read
#pragma unroll
  for (int q = 0; q < 4; ++q) red[q][w][lane] = acc[q];
  __syncthreads();
  if (lv.reduce && w < 4 && own_x) {
    const long long level = lv.t1 + 1;
    kb.partials[(level & 3) * lv.part_stride + ((long long)w * lv.nrt + by) * kp.pitch + x] =
        wave_column_sum(red, w, lane, 1, kR2);
  }
}

// Block b of a two-level launch of one channel (lead blocks, then tiles),
// with the kernel's LDS.
template <class MD, bool NT>
__device__ __forceinline__ void sweep2_block(const KParams& kp, const KBufs& kb, const Lv2& lv,
                                             const typename MD::St* __restrict__ src,
                                             typename MD::St* __restrict__ dst, int b,
                                             typename MD::Pt (*lds)[9][kTX], double (*red)[kW2][kTX],
                                             typename MD::Ct (*pulled)[kStripRowsOf<MD>][9][2], double* kv) {
  constexpr int kRows = kStripRowsOf<MD>;
  double (*redk)[kTY][kTX] = reinterpret_cast<double (*)[kTY][kTX]>(&red[0][0][0]);
  if (b < lv.lead) {
    // the inlet block is block 0 (in a launch of this channel alone on XCD 0,
    // with the first column strips), the outlet block block 7 (XCD 7, with the
    // last ones); the other lead blocks reduce, in order
    if (b == 0 || b == 7) {
      if (!(kp.flags & LBSEP_PERIODIC_X))
        end_block2<MD, NT>(kp, kb, lv, src, dst, b == 7, red, redk,
                           reinterpret_cast<typename MD::Pt (*)[kRows][9]>(&lds[0][0][0]), pulled, kv);
      return;
    }
    const int r = b < 7 ? b - 1 : b - 2;
    constexpr int kWaves = kT2 / kTX;
    const int nsb = strip_blocks(2 * kp.nxt, kWaves);
    if (r < nsb) {
      // strip reductions, one wavefront per task = (level, strip)
      const int task = r * kWaves + int(threadIdx.x / kTX);
      const int li = task / kp.nxt, bx = task - li * kp.nxt;
      // selects, not an index by li: in the batch kernel lv is a local copy,
      // which a dynamic index would move to scratch memory
      const long long level = li == 0 ? lv.strip[0] : (li == 1 ? lv.strip[1] : -1);
      const bool last = li == 1 || lv.strip[1] < 0;  // the latest level keeps the column sums
      if (level >= 0) strip_reduce(kp, kb, bx, level, int(level & 3), lv.nrt, lv.part_stride, 4, last);
    } else if (r == nsb) {
      // the records of up to two levels by one wavefront, in level order: a
      // history ring of one slot keeps the later one
      if (threadIdx.x < kTX)
        for (int k = 0; k < 2; ++k)
          if (lv.glob[k] >= 0) global_reduce(kp, kb, lv.glob[k], int(lv.glob[k] & 3));
    }
    return;
  }
  tile2<MD, NT>(kp, kb, lv, src, dst, b, lds, red);
}

// The LDS of a two-level launch: the tile's first level (or an end block's
// strip), the reduction scratch, the lane-pair end blocks' inner layers and
// the kappa values.
#define LBSEP_SWEEP2_LDS                                                                               \
  constexpr int kRows = kStripRowsOf<MD>;                                                              \
  __shared__ typename MD::Pt lds[kW2][9][kTX];                                                         \
  __shared__ double red[4][kW2][kTX];                                                                  \
  __shared__ typename MD::Ct pulled[kPairEnd<MD> ? 2 : 1][kPairEnd<MD> ? kRows : 1][9][2];             \
  __shared__ double kv[4 * kRows];                                                                     \
  static_assert(4 * kRows * 9 <= kW2 * 9 * kTX, "the end strip fits the tile's LDS");                 \
  auto* pulled_rows = reinterpret_cast<typename MD::Ct (*)[kRows][9][2]>(&pulled[0][0][0][0]);

template <class MD, bool NT>
__global__ __launch_bounds__(kT2) void k_sweep2(const KParams* __restrict__ kpp, const KBufs* __restrict__ kbp, Lv2 lv,
                                                const typename MD::St* __restrict__ src,
                                                typename MD::St* __restrict__ dst) {
  LBSEP_SWEEP2_LDS
  sweep2_block<MD, NT>(*kpp, *kbp, lv, src, dst, (int)blockIdx.x, lds, red, pulled_rows, kv);
}

// A batch of two-level channels swept by one launch per one or two levels:
// entry i holds channel i's constants (its workspace copies), state buffers
// and tiling. The grid is ordered as the one-level batch's (blk_ref), with
// each member's tiles starting at a multiple of 8 blocks, so that its blocks
// keep the XCDs of a launch of that channel alone.
struct Batch2Entry {
  const KParams* kp;
  const KBufs* kb;
  void* f[2];         // the channel's two state buffers
  long long t0;       // channel level at the batch's creation (no reduction pending then)
  int cur0;           // buffer holding the post-collision state at creation
  Lv2 lv;             // tiling; the levels are set per launch
};

// The batch's progress on the device, advanced after each launch
// (k_batch2_advance), so that a captured step loop replays.
struct Batch2Levels {
  long long done;      // levels advanced since creation
  long long launches;  // launches since creation
  int prev_n;          // levels of the previous launch (0: none)
  int prev2_n;         // levels of the launch before it
};

// One launch of nlev levels for every member: levels t0 + done + 1 ..; the
// previous launch's levels are strip-reduced and the one's before reduced to
// records (the order of lbsep_step's two-level launches).
template <class MD, bool NT>
__global__ __launch_bounds__(kT2) void k_sweep2_batch(const Batch2Entry* __restrict__ tab,
                                                      const int2* __restrict__ blk_ref,
                                                      const Batch2Levels* __restrict__ bl, int nlev) {
  LBSEP_SWEEP2_LDS
  using S = typename MD::St;
  const int2 ref = blk_ref[blockIdx.x];
  if (ref.y < 0) return;  // filler before a member's tiles (uniform over the block)
  const Batch2Entry& e = tab[ref.x];
  const long long base = e.t0 + bl->done;  // the members' current level
  const int pn = bl->prev_n, pn2 = bl->prev2_n;
  Lv2 lv = e.lv;
  lv.t1 = base + 1;
  lv.nlev = nlev;
  lv.reduce = 1;
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    lv.strip[k] = k < pn ? base - pn + 1 + k : -1;
    lv.glob[k] = k < pn2 ? base - pn - pn2 + 1 + k : -1;
  }
  const int c = (e.cur0 + (int)(bl->launches & 1)) & 1;
  sweep2_block<MD, NT>(*e.kp, *e.kb, lv, static_cast<const S*>(e.f[c]), static_cast<S*>(e.f[c ^ 1]),
                       ref.y, lds, red, pulled_rows, kv);
}

__global__ void k_batch2_advance(Batch2Levels* bl, int nlev) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    bl->done += nlev;
    bl->launches += 1;
    bl->prev2_n = bl->prev_n;
    bl->prev_n = nlev;
  }
}

__global__ __launch_bounds__(kTX * 8) void k_finalize(KParams kp, KBufs kb, long long t, long long t_first,
                                                       int phase) {
  const int b = blockIdx.x;
  if (phase == 0) {
    const int waves = int(blockDim.x / kTX);  // the channel's sweep block: one strip per wavefront
    if (b < strip_blocks(kp.nxt, waves)) {
      const int bx = b * waves + int(threadIdx.x / kTX);
      if (bx < kp.nxt) strip_reduce(kp, kb, bx, t, int(t & 1), kp.nrt, kb.part_stride, 2);
    } else if (t - 1 >= t_first && threadIdx.x < kTX)
      global_reduce(kp, kb, t - 1, int((t - 1) & 1));
  } else if (phase == 1) {
    if (threadIdx.x < kTX) global_reduce(kp, kb, t, int(t & 1));
  } else {
    // momentum column sums of level t from an evaluation sweep's partials
    const int bx = b * int(blockDim.x / kTX) + int(threadIdx.x / kTX);
    if (bx < kp.nxt) jsum_reduce(kp, kb, bx, int((t + 1) & 1));
  }
}

// Initial state: f = f^eq(rho_s(x), u = 0) (Eq. (feq) at rest), pressure and
// C_l linear in x from (P_in, C_in) to (P_out, C_out); deviation modes store
// f - f0(x).
template <class MD>
__global__ __launch_bounds__(kThreads) void k_init(KParams kp, typename MD::St* __restrict__ f, double p_in,
                                                   double p_out, double c_in, double c_out) {
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
      double fi[9];
      fi[0] = 4.0 / 9.0 * rho[s] * a0;
      for (int i = 1; i < 5; ++i) fi[i] = 1.0 / 9.0 * rho[s] * sv;
      for (int i = 5; i < 9; ++i) fi[i] = 1.0 / 36.0 * rho[s] * sv;
      const double r0 = ref_rho(kp, s, x);
#pragma unroll
      for (int i = 0; i < 9; ++i)
        f[pidx(kp, s, i, j, x)] = typename MD::St(MD::kDev ? fi[i] - kp.wa[s][i] * r0 : fi[i]);
    }
  }
}

// psi(alpha) and psi'(alpha)/2 of the device wall function, element-wise
// (FP64: from the piecewise polynomials if `table`, else the series form).
template <typename T>
__global__ void k_wall_function(const double* __restrict__ a, double* __restrict__ psi, double* __restrict__ h,
                                long long n, int table) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    T p, hh;
    wall_psi<T>(T(a[i]), p, hh, table != 0);
    psi[i] = double(p);
    if (h) h[i] = double(hh);
  }
}

// Volume flow through each cross-section, Q_v(x) = sum_j u_x(x, j) (mixture
// velocity; the species momenta of Eq. (rhou) add up to the mixture momentum),
// from the moment fields [6][ny][nx]; one thread per column, rows in order.
__global__ void k_volume_flow(const double* __restrict__ mom, int nx, int ny, double* __restrict__ q) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= nx) return;
  const long long n = (long long)nx * ny;
  double acc = 0.0;
  for (int j = 0; j < ny; ++j) {
    const long long o = (long long)j * nx + x;
    const double ra = mom[o], rb = mom[n + o];
    acc += (ra * mom[2 * n + o] + rb * mom[4 * n + o]) / (ra + rb);
  }
  q[x] = acc;
}

__global__ void k_zero_u32(unsigned* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

// Dense [2][9][ny][nx] raw state -> state buffer layout.
template <typename S>
__global__ void k_copy_in(KParams kp, const S* __restrict__ dense, S* __restrict__ f) {
  const long long n = 18LL * kp.ny * kp.nx;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (long long)gridDim.x * blockDim.x) {
    const long long row = e / kp.nx;
    const int x = int(e - row * kp.nx);
    const int si = int(row / kp.ny);  // s * 9 + i
    const int j = int(row - (long long)si * kp.ny);
    const int s = si / 9, i = si - 9 * s;
    f[pidx(kp, s, i, j, x)] = dense[e];
  }
}

// Post-collision state (storage representation) -> dense [2][9][ny][nx] FP64
// populations: the stored value, plus f0 of the node's column for deviations.
template <class MD>
__global__ void k_copy_post(KParams kp, const typename MD::St* __restrict__ f, double* __restrict__ dense) {
  const long long n = 18LL * kp.ny * kp.nx;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (long long)gridDim.x * blockDim.x) {
    const long long row = e / kp.nx;
    const int x = int(e - row * kp.nx);
    const int si = int(row / kp.ny);  // s * 9 + i
    const int j = int(row - (long long)si * kp.ny);
    const int s = si / 9, i = si - 9 * s;
    const double v = double(f[pidx(kp, s, i, j, x)]);
    dense[e] = MD::kDev ? v + kp.wa[s][i] * ref_rho(kp, s, x) : v;
  }
}

// Dense [2][9][ny][nx] FP64 populations -> pitched storage representation.
template <class MD>
__global__ void k_set_pop(KParams kp, const double* __restrict__ dense, typename MD::St* __restrict__ f) {
  const long long n = 18LL * kp.ny * kp.nx;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (long long)gridDim.x * blockDim.x) {
    const long long row = e / kp.nx;
    const int x = int(e - row * kp.nx);
    const int si = int(row / kp.ny);  // s * 9 + i
    const int j = int(row - (long long)si * kp.ny);
    const int s = si / 9, i = si - 9 * s;
    const double v = MD::kDev ? dense[e] - kp.wa[s][i] * ref_rho(kp, s, x) : dense[e];
    f[pidx(kp, s, i, j, x)] = typename MD::St(v);
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

size_t elem_bytes(int dtype) { return dtype == LBSEP_F64 ? 8 : dtype == LBSEP_F32 ? 4 : 2; }

struct Layout {
  int pitch, nxt, ntx, nrt, rpt, waves, tiles, lead, nend, nendb;
  bool split;
  bool big;  // a state buffer exceeds half the last-level cache: row-major tiles, non-temporal stores
  bool two;  // two time levels per launch (k_sweep2)
  int ntx2, nrt2, tiles2, chunk2, lead2;
  size_t elem, state_buf, f0, f1, f2, partials, endsum, colsum, strip, hist, status, mom, consts, total;
};

bool validate(const lbsep_params* p, std::string& why) {
  if (!p) return why = "params is NULL", false;
  const bool px = p->flags & LBSEP_PERIODIC_X;
  const bool py = p->flags & LBSEP_PERIODIC_Y;
  if (p->flags & ~0xFu) return why = "unknown flag bits", false;
  if (p->nx < (px ? 1 : 6)) return why = "nx must be >= 6 (>= 1 with LBSEP_PERIODIC_X)", false;
  if (p->ny < 2) return why = "ny must be >= 2", false;
  if ((long long)p->nx * p->ny > (1LL << 31)) return why = "nx * ny too large", false;
  if (p->dtype >= LBSEP_F64 && p->dtype <= LBSEP_F16 &&
      18LL * (long long)align_up((size_t)p->nx, kTX) * (long long)elem_bytes(p->dtype) >= (1LL << 32))
    return why = "channel too long: one row of a state buffer must stay below 4 GiB", false;
  if (p->ny > 64 * kMaxEnd) return why = "ny must be <= " + std::to_string(64 * kMaxEnd), false;
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
  if (p->dtype != LBSEP_F64 && p->dtype != LBSEP_F32 && p->dtype != LBSEP_F16)
    return why = "dtype must be LBSEP_F64, LBSEP_F32 or LBSEP_F16", false;
  if (p->hist_cap < 1) return why = "hist_cap must be >= 1", false;
  if (p->tile_mode < LBSEP_TILE_AUTO || p->tile_mode > LBSEP_TILE_NODE) return why = "bad tile_mode", false;
  if (p->tile_rows != 0 && p->tile_rows != 1 && p->tile_rows != 2 && p->tile_rows != 4)
    return why = "tile_rows must be 0, 1, 2 or 4", false;
  if (p->fused_steps < 0 || p->fused_steps > 2) return why = "fused_steps must be 0, 1 or 2", false;
  if (p->fused_steps == 2 && (px || py)) return why = "fused_steps = 2 needs an inlet, an outlet and walls", false;
  if (p->fused_steps == 2 && p->ny > strip_max_rows(p->dtype))
    return why = std::string("fused_steps = 2 needs ny <= ") +
                 (p->dtype == LBSEP_F64 ? "64 in FP64" : "128 with deviation storage"), false;
  return true;
}

// FP64 channels of more than 2^17 nodes evaluate the wall function from its
// piecewise polynomials, smaller ones (whose steps are latency-bound when they
// run alone) from its series form; a channel keeps its choice in every kernel.
bool wall_psi_table(const lbsep_params* p) {
  return p->dtype == LBSEP_F64 && (long long)p->nx * p->ny > (1LL << 17);
}

Layout make_layout(const lbsep_params* p) {
  Layout L{};
  L.elem = elem_bytes(p->dtype);
  L.pitch = (int)align_up((size_t)p->nx, kTX);
  L.nxt = (p->nx + kTX - 1) / kTX;
  // Tile shape: a lane pair per node (species split) halves each lane's chain,
  // which pays where one wave per SIMD or less is available (latency-bound
  // small channels); one lane per node does less work per node, which pays
  // when the channel fills the GPU many times over.
  if (p->tile_mode == LBSEP_TILE_SPLIT)
    L.split = true;
  else if (p->tile_mode == LBSEP_TILE_NODE)
    L.split = false;
  else  // measured crossover, every dtype: between 61k and 82k nodes
    L.split = (long long)p->nx * p->ny <= (1LL << 16);
  const int cols = L.split ? 32 : 64;
  L.ntx = (p->nx + cols - 1) / cols;
  L.waves = waves_of(p->dtype);
  // rows per thread: as asked, else 4 if that still gives >= 2048 tiles, 2 if
  // >= 512, else 1 (a channel alone needs the parallelism; in a batch that
  // fills the GPU, more rows cut the row-tile partial sums). FP32 stops at 2:
  // measured 2.4-7% faster than 4 on 2.9M-21M-node channels, where FP16 and
  // FP64 are as fast or faster with 4. Two rows at 640-1440 tiles: 1-3.4%
  // faster than one in every dtype; at 360 tiles FP64 loses a fifth.
  L.rpt = 1;
  if (p->tile_rows > 0) {
    L.rpt = p->tile_rows;
  } else {
    for (int r : {4, 2}) {
      if (r == 4 && p->dtype == LBSEP_F32) continue;
      const int nrt = (p->ny + L.waves * r - 1) / (L.waves * r);
      if ((long long)L.ntx * nrt >= (r == 4 ? 2048 : 512)) {
        L.rpt = r;
        break;
      }
    }
  }
  L.nrt = (p->ny + L.waves * L.rpt - 1) / (L.waves * L.rpt);
  L.tiles = L.ntx * L.nrt;
  L.nend = (p->ny + 63) / 64;
  // blocks of 8 wavefronts hold two 64-row units: both ends of a channel of
  // at most 64 rows, else two units of one end
  L.nendb = L.waves == 8 ? (p->ny <= 64 ? 1 : 2 * ((p->ny + 127) / 128)) : 2 * L.nend;
  L.lead = L.nendb + strip_blocks(L.nxt, L.waves) + 1;
  L.state_buf = align_up(18ull * p->ny * L.pitch * L.elem, 256);
  L.big = !L.split && L.state_buf > (128ull << 20);
  // two levels per launch: tiles own 62 columns x 6 rows of the interior
  L.two = p->fused_steps == 2;
  // tiles own columns kEndCols .. nx - 1 - kEndCols; the end blocks the rest
  L.ntx2 = std::max(0, (p->nx - 2 * kEndCols + kC2 - 1) / kC2);
  L.nrt2 = (p->ny + kR2 - 1) / kR2;
  L.tiles2 = L.ntx2 * L.nrt2;
  L.chunk2 = (L.tiles2 + 7) / 8;
  L.lead2 = (int)align_up((size_t)(2 + strip_blocks(2 * L.nxt, kT2 / kTX) + 1), 8);
  size_t off = 0;
  L.f0 = off;
  off += L.state_buf;
  L.f1 = off;
  off += L.state_buf;
  L.f2 = off;  // the level replayed for readouts after a two-level launch
  if (L.two) off += L.state_buf;
  // reduction buffers: two slots (by level parity) for single-level launches,
  // four (level mod 4) for two-level launches
  L.partials = off;
  off += align_up(std::max(2ull * 4 * L.nrt, L.two ? 4ull * 4 * L.nrt2 : 0ull) * L.pitch * sizeof(double), 256);
  L.endsum = off;
  off += align_up(4ull * 2 * kMaxEnd * 4 * sizeof(double), 256);
  L.colsum = off;
  off += align_up(4ull * L.pitch * sizeof(double), 256);
  L.strip = off;
  off += align_up(4ull * 4 * L.nxt * sizeof(double), 256);
  L.hist = off;
  off += align_up(4ull * p->hist_cap * sizeof(double), 256);
  L.status = off;
  off += 256;
  L.mom = off;
  off += align_up(6ull * p->ny * p->nx * sizeof(double), 256);
  L.consts = off;  // copies of KParams and KBufs, the two-level kernel's constants
  off += align_up(sizeof(KParams), 256) + align_up(sizeof(KBufs), 256);
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
  int cur;          // buffer holding f'(t)
  bool prev_pre;    // the other buffer holds the pre-collision f(t) (after init / set_state)
  int64_t t;
  int64_t t_first;  // first level with a history record
  bool finalized;   // records of levels t-1 and t are complete
  // two levels per launch
  void* f2;           // third state buffer
  int prev_buf;       // buffer holding f'(t-1) for readouts: 0, 1, 2 (f2), -1: not held (replay first)
  int64_t strip_next;  // levels below are strip-reduced
  int64_t glob_next;   // levels below have their record
  bool pipe2;          // levels since the last set / init came from two-level launches
  uint64_t gen;        // bumped by every change of the state (init, set, step): batches check it
};

namespace {

int check_hip(hipError_t e, const char* what) {
  if (e != hipSuccess) return fail(LBSEP_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
  return LBSEP_OK;
}

template <class MD, bool PULL, bool EVAL>
void launch_sweep(lbsep_channel* h, const void* src, void* dst, double* mom, void* fraw, double* ffull,
                  long long t, int jsums) {
  using S = typename MD::St;
  const int grid = h->L.lead + h->L.tiles;
  if (h->L.split)
    hipLaunchKernelGGL((k_sweep<MD, PULL, EVAL, true, false>), dim3(grid), dim3(kTX * kWaves<MD>), 0, h->stream, h->kp,
                       h->kb, static_cast<const S*>(src), static_cast<S*>(dst), mom, static_cast<S*>(fraw), ffull, t,
                       (long long)h->t_first, jsums);
  else if (h->L.big && !EVAL)
    hipLaunchKernelGGL((k_sweep<MD, PULL, EVAL, false, true>), dim3(grid), dim3(kTX * kWaves<MD>), 0, h->stream, h->kp,
                       h->kb, static_cast<const S*>(src), static_cast<S*>(dst), mom, static_cast<S*>(fraw), ffull, t,
                       (long long)h->t_first, jsums);
  else
    hipLaunchKernelGGL((k_sweep<MD, PULL, EVAL, false, false>), dim3(grid), dim3(kTX * kWaves<MD>), 0, h->stream, h->kp,
                       h->kb, static_cast<const S*>(src), static_cast<S*>(dst), mom, static_cast<S*>(fraw), ffull, t,
                       (long long)h->t_first, jsums);
}

template <bool PULL, bool EVAL>
void sweep_any(lbsep_channel* h, const void* src, void* dst, double* mom, void* fraw, double* ffull, long long t,
               int jsums = 0) {
  switch (h->p.dtype) {
    case LBSEP_F64:
      if (h->kp.rc.psi_table)
        launch_sweep<PsiMode<ModeF64, 2>, PULL, EVAL>(h, src, dst, mom, fraw, ffull, t, jsums);
      else
        launch_sweep<PsiMode<ModeF64, 1>, PULL, EVAL>(h, src, dst, mom, fraw, ffull, t, jsums);
      break;
    case LBSEP_F32:
      launch_sweep<ModeF32, PULL, EVAL>(h, src, dst, mom, fraw, ffull, t, jsums);
      break;
    default:
      launch_sweep<ModeF16, PULL, EVAL>(h, src, dst, mom, fraw, ffull, t, jsums);
      break;
  }
}

template <class MD>
void launch_sweep2_md(lbsep_channel* h, const Lv2& lv, int grid, const void* src, void* dst) {
  using S = typename MD::St;
  // non-temporal state stores at every size, also where the state fits the
  // caches (64x1280: FP64 11.50 vs 11.76 us per level, FP32 5.38 vs 5.42)
  hipLaunchKernelGGL((k_sweep2<MD, true>), dim3(grid), dim3(kT2), 0, h->stream,
                     reinterpret_cast<const KParams*>(h->ws + h->L.consts),
                     reinterpret_cast<const KBufs*>(h->ws + h->L.consts + align_up(sizeof(KParams), 256)), lv,
                     static_cast<const S*>(src), static_cast<S*>(dst));
}

// k_sweep2 over the whole grid, or (nlev == 0) its lead blocks only.
void launch_sweep2(lbsep_channel* h, const Lv2& lv, const void* src, void* dst) {
  const int grid = lv.nlev == 0 ? lv.lead : lv.lead + 8 * lv.chunk;
  const bool tall = h->p.ny > 64;
  switch (h->p.dtype) {
    case LBSEP_F64:
      launch_sweep2_md<StripMode<ModeF64, 64>>(h, lv, grid, src, dst);
      break;
    case LBSEP_F32:
      if (tall)
        launch_sweep2_md<StripMode<ModeF32, 128>>(h, lv, grid, src, dst);
      else
        launch_sweep2_md<StripMode<ModeF32, 64>>(h, lv, grid, src, dst);
      break;
    default:
      if (tall)
        launch_sweep2_md<StripMode<ModeF16, 128>>(h, lv, grid, src, dst);
      else
        launch_sweep2_md<StripMode<ModeF16, 64>>(h, lv, grid, src, dst);
      break;
  }
}

// Arguments of a k_sweep2 launch computing nlev levels from t1 on, with empty
// level lists.
Lv2 sweep2_args(const lbsep_channel* h, long long t1, int nlev, int reduce) {
  const Layout& L = h->L;
  Lv2 lv{};
  lv.ntx = L.ntx2;
  lv.nrt = L.nrt2;
  lv.tiles = L.tiles2;
  lv.chunk = L.chunk2;
  lv.lead = L.lead2;
  lv.part_stride = 4LL * L.nrt2 * L.pitch;
  lv.t1 = t1;
  lv.nlev = nlev;
  lv.reduce = reduce;
  lv.strip[0] = lv.strip[1] = lv.glob[0] = lv.glob[1] = -1;
  return lv;
}

// Level lists of a two-level launch: strip-reduce the levels not yet
// strip-reduced, reduce to records those strip-reduced before.
Lv2 pending_levels(const lbsep_channel* h, int nlev, int reduce) {
  Lv2 lv = sweep2_args(h, h->t + 1, nlev, reduce);
  int k = 0;
  for (int64_t l = h->strip_next; l <= h->t && k < 2; ++l) lv.strip[k++] = l;
  k = 0;
  for (int64_t l = h->glob_next; l < h->strip_next && k < 2; ++l) lv.glob[k++] = l;
  return lv;
}

int finalize(lbsep_channel* h);

// Collide the pre-collision state held in f[0] into f[1] at level t.
int collide_loaded(lbsep_channel* h, int64_t t) {
  ++h->gen;
  h->t_first = t;
  sweep_any<false, false>(h, h->f[0], h->f[1], nullptr, nullptr, nullptr, t);
  h->cur = 1;
  h->prev_pre = true;
  h->prev_buf = 0;
  h->t = t;
  h->finalized = false;
  h->pipe2 = false;
  int rc = check_hip(hipGetLastError(), "collide launch");
  if (rc == LBSEP_OK && h->L.two) {
    // complete the record of level t with the single-level reductions, so the
    // two-level pipeline starts with nothing pending
    rc = finalize(h);
    h->strip_next = h->glob_next = t + 1;
  }
  return rc;
}

// Complete the records of the last levels (idempotent).
int finalize(lbsep_channel* h) {
  if (h->finalized) return LBSEP_OK;
  if (h->pipe2) {
    Lv2 lv = pending_levels(h, 0, 0);
    launch_sweep2(h, lv, nullptr, nullptr);
    h->glob_next = h->strip_next;
    h->strip_next = h->t + 1;
    lv = pending_levels(h, 0, 0);
    launch_sweep2(h, lv, nullptr, nullptr);
    h->glob_next = h->strip_next;
  } else {
    hipLaunchKernelGGL(k_finalize, dim3(strip_blocks(h->L.nxt, h->L.waves) + 1), dim3(kTX * h->L.waves), 0, h->stream,
                       h->kp, h->kb,
                       (long long)h->t, (long long)h->t_first, 0);
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kTX * h->L.waves), 0, h->stream, h->kp, h->kb, (long long)h->t,
                       (long long)h->t_first, 1);
  }
  h->finalized = true;
  return check_hip(hipGetLastError(), "finalize launch");
}

// EVAL sweep of the current state into mom, fraw and/or ffull.
int eval_state(lbsep_channel* h, double* mom, void* fraw, double* ffull, int jsums = 0) {
  if (h->prev_buf < 0) {
    // the last launch advanced two levels: recompute f'(t-1) from f'(t-2)
    // (held by the other buffer) into f2, without reductions
    launch_sweep2(h, sweep2_args(h, h->t - 1, 1, 0), h->f[1 - h->cur], h->f2);
    h->prev_buf = 2;
  }
  const void* prev = h->prev_buf == 2 ? h->f2 : h->f[h->prev_buf];
  if (h->prev_pre)
    sweep_any<false, true>(h, prev, nullptr, mom, fraw, ffull, h->t, jsums);
  else
    sweep_any<true, true>(h, prev, nullptr, mom, fraw, ffull, h->t, jsums);
  return check_hip(hipGetLastError(), "eval launch");
}

template <class MD>
void launch_init(lbsep_channel* h, double p_in, double p_out) {
  const int igrid = (int)std::min<long long>(4096, ((long long)h->p.ny * h->L.pitch + 255) / 256);
  hipLaunchKernelGGL(k_init<MD>, dim3(igrid), dim3(kThreads), 0, h->stream, h->kp,
                     static_cast<typename MD::St*>(h->f[0]), p_in, p_out, h->p.cl_in, h->p.cl_out);
}

template <class MD>
void launch_set_pop(lbsep_channel* h, const double* src) {
  hipLaunchKernelGGL(k_set_pop<MD>, dim3(2048), dim3(256), 0, h->stream, h->kp, src,
                     static_cast<typename MD::St*>(h->f[0]));
}

// A recording step of an FP64 channel (MD: its wall-function evaluation).
template <class MD>
void launch_record(lbsep_channel* h, int grid, const double* src, double* dst, double* dev_pre, double* dev_post) {
  if (h->L.split)
    hipLaunchKernelGGL((k_sweep<MD, true, false, true, false, true>), dim3(grid), dim3(kTX * kWaves<MD>), 0, h->stream,
                       h->kp, h->kb, src, dst, nullptr, dev_post, dev_pre, (long long)(h->t + 1),
                       (long long)h->t_first, 0);
  else
    hipLaunchKernelGGL((k_sweep<MD, true, false, false, false, true>), dim3(grid), dim3(kTX * kWaves<MD>), 0,
                       h->stream, h->kp, h->kb, src, dst, nullptr, dev_post, dev_pre, (long long)(h->t + 1),
                       (long long)h->t_first, 0);
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
  return 18ull * p->ny * p->nx * elem_bytes(p->dtype);
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
  if (ws_bytes < L.total) return fail(LBSEP_ESIZE, "workspace too small: need " + std::to_string(L.total) + " bytes");
  lbsep_channel* h = new (std::nothrow) lbsep_channel();
  if (!h) return fail(LBSEP_EDEVICE, "out of host memory");
  h->p = *p;
  h->L = L;
  h->stream = static_cast<hipStream_t>(hip_stream);
  h->ws = static_cast<char*>(dev_ws);
  h->f[0] = h->ws + L.f0;
  h->f[1] = h->ws + L.f1;
  h->f2 = L.two ? h->ws + L.f2 : nullptr;
  h->mom = reinterpret_cast<double*>(h->ws + L.mom);

  KParams& kp = h->kp;
  const bool px = p->flags & LBSEP_PERIODIC_X;
  const double m_min = p->m_a;  // validated: m_a <= m_b
  const double cs2 = 1.0 / 3.0, p_out = cs2, p_in = p->theta * cs2;
  kp.nx = p->nx;
  kp.ny = p->ny;
  kp.pitch = L.pitch;
  kp.nxt = L.nxt;
  kp.nrt = L.nrt;
  kp.ntx = L.ntx;
  kp.rpt = L.rpt;
  kp.tiles = L.tiles;
  kp.lead = L.lead;
  kp.nend = L.nend;
  kp.nendb = L.nendb;
  kp.row = 18LL * L.pitch;
  kp.flags = p->flags | (h->L.split ? 0u : kRowMajorTiles);
  kp.r = p->dbb_r;
  kp.cl_in = p->cl_in;
  RelaxConsts& rc = kp.rc;
  rc.inv_m[0] = 1.0 / p->m_a;
  rc.inv_m[1] = 1.0 / p->m_b;
  rc.s[0] = m_min / p->m_a;
  rc.s[1] = m_min / p->m_b;
  rc.lam_p = p->kn_out * double(p->ny) * p_out;
  rc.inv_lam_p = 1.0 / rc.lam_p;
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
  rc.psi_table = wall_psi_table(p) ? 1 : 0;
  // species densities at the ends: rho_s = x_s P / (s_s c_s^2)
  kp.rho_bc[0][0] = p->cl_in * p_in / (rc.s[0] * cs2);
  kp.rho_bc[0][1] = (1.0 - p->cl_in) * p_in / (rc.s[1] * cs2);
  kp.rho_bc[1][0] = p->cl_out * p_out / (rc.s[0] * cs2);
  kp.rho_bc[1][1] = (1.0 - p->cl_out) * p_out / (rc.s[1] * cs2);
  // reference density of the deviation modes and the lattice weights w_i alpha_si
  static const double w[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
  static const int cx[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
  for (int s = 0; s < 2; ++s) {
    kp.ref0[s] = kp.rho_bc[0][s];
    kp.slope[s] = px ? 0.0 : (kp.rho_bc[1][s] - kp.rho_bc[0][s]) / double(p->nx - 1);
    for (int i = 0; i < 9; ++i) {
      kp.wa[s][i] = w[i] * (i == 0 ? (9.0 - 5.0 * rc.s[s]) / 4.0 : rc.s[s]);
      kp.corr[s][i] = -double(cx[i]) * kp.wa[s][i] * kp.slope[s];
    }
  }

  KBufs& kb = h->kb;
  kb.partials = reinterpret_cast<double*>(h->ws + L.partials);
  kb.endsum = reinterpret_cast<double*>(h->ws + L.endsum);
  kb.colsum = reinterpret_cast<double*>(h->ws + L.colsum);
  kb.strip = reinterpret_cast<double*>(h->ws + L.strip);
  kb.hist = reinterpret_cast<double*>(h->ws + L.hist);
  kb.status = reinterpret_cast<unsigned*>(h->ws + L.status);
  kb.hist_cap = p->hist_cap;
  kb.part_stride = 4LL * L.nrt * L.pitch;

  // the two-level kernel reads KParams and KBufs from this copy: a launch
  // with a few hundred bytes less of arguments starts about 1.7 us sooner.
  // Enqueued before every kernel of the channel; the sources live in the
  // channel and never change, so nothing waits here.
  if (hipMemcpyAsync(h->ws + L.consts, &h->kp, sizeof(KParams), hipMemcpyHostToDevice, h->stream) != hipSuccess ||
      hipMemcpyAsync(h->ws + L.consts + align_up(sizeof(KParams), 256), &h->kb, sizeof(KBufs), hipMemcpyHostToDevice,
                     h->stream) != hipSuccess) {
    delete h;
    return fail(LBSEP_EDEVICE, "copying the kernel constants");
  }
  hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(256), 0, h->stream, kb.status, 1);
  switch (p->dtype) {
    case LBSEP_F64:
      launch_init<ModeF64>(h, p_in, p_out);
      break;
    case LBSEP_F32:
      launch_init<ModeF32>(h, p_in, p_out);
      break;
    default:
      launch_init<ModeF16>(h, p_in, p_out);
      break;
  }
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
  if (nsteps > 0) ++h->gen;
  if (h->L.two) {
    for (int64_t n = nsteps; n > 0;) {
      const int nlev = n >= 2 ? 2 : 1;
      const int nxt_buf = 1 - h->cur;
      const Lv2 lv = pending_levels(h, nlev, 1);
      launch_sweep2(h, lv, h->f[h->cur], h->f[nxt_buf]);
      h->pipe2 = true;
      h->glob_next = h->strip_next;
      h->strip_next = h->t + 1;
      h->prev_buf = nlev == 2 ? -1 : h->cur;
      h->cur = nxt_buf;
      h->prev_pre = false;
      h->t += nlev;
      h->finalized = false;
      n -= nlev;
    }
    return check_hip(hipGetLastError(), "step launch");
  }
  for (int64_t n = 0; n < nsteps; ++n) {
    const int nxt_buf = 1 - h->cur;
    sweep_any<true, false>(h, h->f[h->cur], h->f[nxt_buf], nullptr, nullptr, nullptr, (long long)(h->t + 1));
    h->prev_buf = h->cur;
    h->cur = nxt_buf;
    h->prev_pre = false;
    h->t += 1;
    h->finalized = false;
  }
  return check_hip(hipGetLastError(), "step launch");
}

int64_t lbsep_time(const lbsep_channel* h) { return h ? h->t : -1; }

int lbsep_step_record(lbsep_channel* h, double* dev_pre, double* dev_post) {
  if (!h) return fail(LBSEP_EINVAL, "channel is NULL");
  if (!dev_pre || !dev_post) return fail(LBSEP_EINVAL, "dev_pre and dev_post must be device pointers");
  if (h->p.dtype != LBSEP_F64) return fail(LBSEP_EINVAL, "lbsep_step_record needs an FP64 channel");
  if (h->L.two) return fail(LBSEP_EINVAL, "lbsep_step_record needs one level per launch (fused_steps 0 or 1)");
  ++h->gen;
  const int nxt_buf = 1 - h->cur;
  const int grid = h->L.lead + h->L.tiles;
  const double* src = static_cast<const double*>(h->f[h->cur]);
  double* dst = static_cast<double*>(h->f[nxt_buf]);
  // the recording variant: ffull <- pulled populations, fraw <- post-collision
  if (h->kp.rc.psi_table)
    launch_record<PsiMode<ModeF64, 2>>(h, grid, src, dst, dev_pre, dev_post);
  else
    launch_record<PsiMode<ModeF64, 1>>(h, grid, src, dst, dev_pre, dev_post);
  h->prev_buf = h->cur;
  h->cur = nxt_buf;
  h->prev_pre = false;
  h->t += 1;
  h->finalized = false;
  return check_hip(hipGetLastError(), "step launch");
}

int lbsep_read_cl(lbsep_channel* h, double* cl, double* cl_tilde, int32_t* x_min, double* profile) {
  if (!h) return fail(LBSEP_EINVAL, "channel is NULL");
  if (int e = finalize(h)) return e;
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
  if (int e = finalize(h)) return e;
  if (!h->pipe2) {
    // one-level launches carry only the density sums: the momentum sums of
    // the current level come from an evaluation sweep and a strip pass
    if (int e = eval_state(h, nullptr, nullptr, nullptr, 1)) return e;
    hipLaunchKernelGGL(k_finalize, dim3(strip_blocks(h->L.nxt, h->L.waves)), dim3(kTX * h->L.waves), 0, h->stream, h->kp, h->kb,
                       (long long)h->t, (long long)h->t_first, 2);
    if (int e = check_hip(hipGetLastError(), "column sums launch")) return e;
  }
  int rc = check_hip(hipMemcpy2DAsync(host, h->p.nx * sizeof(double), h->kb.colsum, h->L.pitch * sizeof(double),
                                      h->p.nx * sizeof(double), 4, hipMemcpyDeviceToHost, h->stream),
                     "column sums copy");
  if (!rc) rc = check_hip(hipStreamSynchronize(h->stream), "column sums sync");
  return rc;
}

int lbsep_read_history(lbsep_channel* h, int64_t t0, int64_t count, double* host) {
  if (!h || (!host && count > 0) || count < 0) return fail(LBSEP_EINVAL, "bad argument");
  if (count == 0) return LBSEP_OK;
  if (int e = finalize(h)) return e;
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
  int rc = eval_state(h, h->mom, nullptr, nullptr);
  if (rc) return rc;
  rc = check_hip(hipMemcpyAsync(host, h->mom, 6ull * h->p.ny * h->p.nx * sizeof(double), hipMemcpyDeviceToHost,
                                h->stream),
                 "moments copy");
  if (!rc) rc = check_hip(hipStreamSynchronize(h->stream), "moments sync");
  return rc;
}

int lbsep_read_volume_flow(lbsep_channel* h, double* host) {
  if (!h || !host) return fail(LBSEP_EINVAL, "NULL argument");
  int rc = eval_state(h, h->mom, nullptr, nullptr);
  if (rc) return rc;
  // the profile is written over the u_ay plane, which the flow does not read
  double* q = h->mom + 3ull * h->p.ny * h->p.nx;
  hipLaunchKernelGGL(k_volume_flow, dim3((h->p.nx + 255) / 256), dim3(256), 0, h->stream, h->mom, h->p.nx,
                     h->p.ny, q);
  rc = check_hip(hipGetLastError(), "volume flow launch");
  if (!rc)
    rc = check_hip(hipMemcpyAsync(host, q, (size_t)h->p.nx * sizeof(double), hipMemcpyDeviceToHost, h->stream),
                   "volume flow copy");
  if (!rc) rc = check_hip(hipStreamSynchronize(h->stream), "volume flow sync");
  return rc;
}

int lbsep_get_state(lbsep_channel* h, void* dev_dst) {
  if (!h || !dev_dst) return fail(LBSEP_EINVAL, "NULL argument");
  return eval_state(h, nullptr, dev_dst, nullptr);
}

int lbsep_get_populations(lbsep_channel* h, double* dev_dst) {
  if (!h || !dev_dst) return fail(LBSEP_EINVAL, "NULL argument");
  return eval_state(h, nullptr, nullptr, dev_dst);
}

int lbsep_get_post_collision(lbsep_channel* h, double* dev_dst) {
  if (!h || !dev_dst) return fail(LBSEP_EINVAL, "NULL argument");
  const void* cur = h->f[h->cur];
  switch (h->p.dtype) {
    case LBSEP_F64:
      hipLaunchKernelGGL(k_copy_post<ModeF64>, dim3(2048), dim3(256), 0, h->stream, h->kp,
                         static_cast<const double*>(cur), dev_dst);
      break;
    case LBSEP_F32:
      hipLaunchKernelGGL(k_copy_post<ModeF32>, dim3(2048), dim3(256), 0, h->stream, h->kp,
                         static_cast<const float*>(cur), dev_dst);
      break;
    default:
      hipLaunchKernelGGL(k_copy_post<ModeF16>, dim3(2048), dim3(256), 0, h->stream, h->kp,
                         static_cast<const _Float16*>(cur), dev_dst);
      break;
  }
  return check_hip(hipGetLastError(), "post-collision copy");
}

int lbsep_set_state(lbsep_channel* h, const void* dev_src, int64_t t) {
  if (!h || !dev_src) return fail(LBSEP_EINVAL, "NULL argument");
  if (t < 0) return fail(LBSEP_EINVAL, "t must be >= 0");
  hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(256), 0, h->stream, h->kb.status, 1);
  switch (h->p.dtype) {
    case LBSEP_F64:
      hipLaunchKernelGGL(k_copy_in<double>, dim3(2048), dim3(256), 0, h->stream, h->kp,
                         static_cast<const double*>(dev_src), static_cast<double*>(h->f[0]));
      break;
    case LBSEP_F32:
      hipLaunchKernelGGL(k_copy_in<float>, dim3(2048), dim3(256), 0, h->stream, h->kp,
                         static_cast<const float*>(dev_src), static_cast<float*>(h->f[0]));
      break;
    default:
      hipLaunchKernelGGL(k_copy_in<_Float16>, dim3(2048), dim3(256), 0, h->stream, h->kp,
                         static_cast<const _Float16*>(dev_src), static_cast<_Float16*>(h->f[0]));
      break;
  }
  int rc = check_hip(hipGetLastError(), "set_state copy");
  if (rc) return rc;
  return collide_loaded(h, t);
}

int lbsep_set_populations(lbsep_channel* h, const double* dev_src, int64_t t) {
  if (!h || !dev_src) return fail(LBSEP_EINVAL, "NULL argument");
  if (t < 0) return fail(LBSEP_EINVAL, "t must be >= 0");
  hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(256), 0, h->stream, h->kb.status, 1);
  switch (h->p.dtype) {
    case LBSEP_F64:
      launch_set_pop<ModeF64>(h, dev_src);
      break;
    case LBSEP_F32:
      launch_set_pop<ModeF32>(h, dev_src);
      break;
    default:
      launch_set_pop<ModeF16>(h, dev_src);
      break;
  }
  int rc = check_hip(hipGetLastError(), "set_populations");
  if (rc) return rc;
  return collide_loaded(h, t);
}

int lbsep_wall_function(const double* dev_alpha, double* dev_psi, double* dev_h, int64_t n, int32_t dtype,
                        int32_t table, void* hip_stream) {
  if (n < 0 || (n > 0 && (!dev_alpha || !dev_psi))) return fail(LBSEP_EINVAL, "bad argument");
  if (dtype != LBSEP_F64 && dtype != LBSEP_F32 && dtype != LBSEP_F16) return fail(LBSEP_EINVAL, "bad dtype");
  if (table != 0 && table != 1) return fail(LBSEP_EINVAL, "bad table");
  if (n == 0) return LBSEP_OK;
  const int grid = (int)std::min<int64_t>(1024, (n + 255) / 256);
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  if (dtype == LBSEP_F64)
    hipLaunchKernelGGL(k_wall_function<double>, dim3(grid), dim3(256), 0, st, dev_alpha, dev_psi, dev_h, (long long)n,
                       (int)table);
  else
    hipLaunchKernelGGL(k_wall_function<float>, dim3(grid), dim3(256), 0, st, dev_alpha, dev_psi, dev_h, (long long)n,
                       (int)table);
  return check_hip(hipGetLastError(), "wall function launch");
}

void lbsep_destroy(lbsep_channel* h) { delete h; }

}  // extern "C"

// ---------------------------------------------------------------------------
// Batches: several channels advanced by one launch per step
// ---------------------------------------------------------------------------
struct lbsep_batch {
  std::vector<lbsep_channel*> ch;
  std::vector<uint64_t> gen_expect;  // member state generations the device table was set up for
  hipStream_t stream = nullptr;
  int dtype = 0;
  bool nt = false;
  int total_blocks = 0;
  long long* counter = nullptr;  // device: batch steps taken
  BatchEntry* tab = nullptr;     // device
  int2* blk_ref = nullptr;       // device: block -> (entry, block of that entry's launch)
  bool two = false;              // members advance two levels per launch (k_sweep2_batch)
  bool tall2 = false;            // a two-level member has more than 64 rows (128-row end strips)
  Batch2Entry* tab2 = nullptr;   // device (two-level members)
  Batch2Levels* lev2 = nullptr;  // device: progress of the two-level launches
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int64_t graph_steps = 0;
};

namespace {

struct BatchLayout {
  size_t counter, tab, blk, total;
  int blocks;
  bool two;
};

// The batch grid (see BatchEntry): every member's end blocks, then every
// member's reduction blocks, then each member's tiles; with two levels per
// launch (end blocks 0 and 7 of a member's lead) each member's tiles start at
// a multiple of 8. Returns the number of blocks; fills refs if not NULL.
long long batch_grid(lbsep_channel* const* chans, int n, bool two, std::vector<int2>* refs) {
  long long k = 0;
  auto put = [&](int i, int b) {
    if (refs) (*refs)[k] = make_int2(i, b);
    ++k;
  };
  for (int i = 0; i < n; ++i) {
    const Layout& L = chans[i]->L;
    if (two) {
      put(i, 0);
      put(i, 7);
    } else {
      for (int b = 0; b < L.nendb; ++b) put(i, b);
    }
  }
  for (int i = 0; i < n; ++i) {
    const Layout& L = chans[i]->L;
    if (two) {
      for (int b = 1; b < L.lead2; ++b)
        if (b != 7) put(i, b);
    } else {
      for (int b = L.nendb; b < L.lead; ++b) put(i, b);
    }
  }
  if (two) {
    for (int i = 0; i < n; ++i) {
      const Layout& L = chans[i]->L;
      while (k & 7) put(i, -1);  // filler block
      for (int b = 0; b < 8 * L.chunk2; ++b) put(i, L.lead2 + b);
    }
    return k;
  }
  // one-level tiles, every member's in its own order, dealt out in runs of
  // kXcdRun per XCD as k_sweep deals a channel's (xcd_run_block)
  std::vector<int2> tl;
  for (int i = 0; i < n; ++i) {
    const Layout& L = chans[i]->L;
    for (int b = 0; b < L.tiles; ++b) tl.push_back(make_int2(i, L.lead + b));
  }
  const size_t grp = 8 * kXcdRun;
  const size_t full = tl.size() / grp * grp;
  for (size_t g = 0; g < full; g += grp)
    for (int t = 0; t < kXcdRun; ++t)
      for (int j = 0; j < 8; ++j) put(tl[g + kXcdRun * j + t].x, tl[g + kXcdRun * j + t].y);
  for (size_t q = full; q < tl.size(); ++q) put(tl[q].x, tl[q].y);
  return k;
}

int batch_layout(lbsep_channel* const* chans, int n, BatchLayout& B) {
  if (!chans || n < 1) return fail(LBSEP_EINVAL, "need at least one channel");
  B.blocks = 0;
  B.two = chans[0] && chans[0]->L.two;
  for (int i = 0; i < n; ++i) {
    if (!chans[i]) return fail(LBSEP_EINVAL, "channel " + std::to_string(i) + " is NULL");
    for (int k = 0; k < i; ++k)
      if (chans[k] == chans[i]) return fail(LBSEP_EINVAL, "a channel appears twice in the batch");
    if (chans[i]->p.dtype != chans[0]->p.dtype) return fail(LBSEP_EINVAL, "all channels of a batch share one dtype");
    if (chans[i]->stream != chans[0]->stream) return fail(LBSEP_EINVAL, "all channels of a batch share one stream");
    if (chans[i]->L.two != B.two)
      return fail(LBSEP_EINVAL, "batch members all advance one level per launch or all two (fused_steps)");
  }
  const long long nb = batch_grid(chans, n, B.two, nullptr);
  if (nb > (1LL << 30)) return fail(LBSEP_EINVAL, "batch grid too large");
  B.blocks = (int)nb;
  size_t off = 0;
  B.counter = off;
  off += 256;
  B.tab = off;
  off += align_up((size_t)n * std::max(sizeof(BatchEntry), sizeof(Batch2Entry)) + sizeof(Batch2Levels), 256);
  B.blk = off;
  off += align_up((size_t)B.blocks * sizeof(int2), 256);
  B.total = off;
  return LBSEP_OK;
}

template <class MD>
void launch_batch(lbsep_batch* b, int k_local) {
  if (b->nt)
    hipLaunchKernelGGL((k_sweep_batch<MD, true>), dim3(b->total_blocks), dim3(kTX * kWaves<MD>), 0, b->stream, b->tab,
                       b->blk_ref, b->counter, k_local);
  else
    hipLaunchKernelGGL((k_sweep_batch<MD, false>), dim3(b->total_blocks), dim3(kTX * kWaves<MD>), 0, b->stream, b->tab,
                       b->blk_ref, b->counter, k_local);
}

template <class MD>
void launch_batch2(lbsep_batch* b, int nlev) {
  hipLaunchKernelGGL((k_sweep2_batch<MD, true>), dim3(b->total_blocks), dim3(kT2), 0, b->stream, b->tab2,
                     b->blk_ref, b->lev2, nlev);
  hipLaunchKernelGGL(k_batch2_advance, dim3(1), dim3(64), 0, b->stream, b->lev2, nlev);
}

// n levels of a two-level batch: launches of two levels, the last of one if
// n is odd; the device record of the progress follows each launch.
void enqueue_batch2_levels(lbsep_batch* b, int64_t n) {
  for (int64_t left = n; left > 0;) {
    const int nlev = left >= 2 ? 2 : 1;
    switch (b->dtype) {
      case LBSEP_F64:
        launch_batch2<StripMode<ModeF64, 64>>(b, nlev);
        break;
      case LBSEP_F32:
        if (b->tall2)
          launch_batch2<StripMode<ModeF32, 128>>(b, nlev);
        else
          launch_batch2<StripMode<ModeF32, 64>>(b, nlev);
        break;
      default:
        if (b->tall2)
          launch_batch2<StripMode<ModeF16, 128>>(b, nlev);
        else
          launch_batch2<StripMode<ModeF16, 64>>(b, nlev);
        break;
    }
    left -= nlev;
  }
}

// n sweeps (k_local = 0 .. n-1 from the current counter), then counter += n.
void enqueue_batch_steps(lbsep_batch* b, int64_t n) {
  if (b->two) {
    enqueue_batch2_levels(b, n);
    return;
  }
  for (int64_t k = 0; k < n; ++k) {
    switch (b->dtype) {
      case LBSEP_F64:
        launch_batch<ModeF64>(b, (int)k);
        break;
      case LBSEP_F32:
        launch_batch<ModeF32>(b, (int)k);
        break;
      default:
        launch_batch<ModeF16>(b, (int)k);
        break;
    }
  }
  hipLaunchKernelGGL(k_batch_advance, dim3(1), dim3(64), 0, b->stream, b->counter, (long long)n);
}

void drop_graph(lbsep_batch* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
  b->graph_steps = 0;
}

}  // namespace

namespace lbsep {

bool channel_view(const lbsep_channel* h, ChannelView* out) {
  if (!h || !out) return false;
  out->p = h->p;
  out->rc = h->kp.rc;
  for (int e = 0; e < 2; ++e)
    for (int s = 0; s < 2; ++s) out->rho_bc[e][s] = h->kp.rho_bc[e][s];
  out->stream = h->stream;
  return true;
}

int set_error(int code, const char* msg) { return fail(code, msg); }

}  // namespace lbsep

extern "C" {

size_t lbsep_batch_workspace_bytes(lbsep_channel* const* chans, int32_t n) {
  BatchLayout B;
  if (batch_layout(chans, n, B)) return 0;
  return B.total;
}

int lbsep_batch_create(lbsep_channel* const* chans, int32_t n, void* dev_ws, size_t ws_bytes, lbsep_batch** out) {
  if (!out) return fail(LBSEP_EINVAL, "out is NULL");
  *out = nullptr;
  BatchLayout B;
  if (int e = batch_layout(chans, n, B)) return e;
  if (!dev_ws || (reinterpret_cast<uintptr_t>(dev_ws) & 255u))
    return fail(LBSEP_EINVAL, "dev_ws must be a non-NULL 256-byte aligned device pointer");
  if (ws_bytes < B.total) return fail(LBSEP_ESIZE, "workspace too small: need " + std::to_string(B.total) + " bytes");
  auto* b = new (std::nothrow) lbsep_batch;
  if (!b) return fail(LBSEP_EDEVICE, "out of host memory");
  char* ws = static_cast<char*>(dev_ws);
  b->stream = chans[0]->stream;
  b->dtype = chans[0]->p.dtype;
  b->counter = reinterpret_cast<long long*>(ws + B.counter);
  b->tab = reinterpret_cast<BatchEntry*>(ws + B.tab);
  b->blk_ref = reinterpret_cast<int2*>(ws + B.blk);
  b->total_blocks = B.blocks;
  b->two = B.two;
  for (int i = 0; i < n; ++i)
    if (chans[i]->p.ny > 64) b->tall2 = true;
  if (B.two) {
    b->tab2 = reinterpret_cast<Batch2Entry*>(ws + B.tab);
    b->lev2 = reinterpret_cast<Batch2Levels*>(ws + B.tab + (size_t)n * sizeof(Batch2Entry));
    // the two-level pipeline starts with nothing pending: every member's
    // records are completed first (enqueued before the table copy)
    for (int i = 0; i < n; ++i)
      if (int e = finalize(chans[i])) {
        delete b;
        return e;
      }
  }
  std::vector<BatchEntry> host(n);
  std::vector<Batch2Entry> host2(B.two ? n : 0);
  std::vector<int2> blk(B.blocks);
  batch_grid(chans, n, B.two, &blk);
  size_t node_state = 0;
  for (int i = 0; i < n && B.two; ++i) {
    lbsep_channel* c = chans[i];
    Batch2Entry& e = host2[i];
    std::memset(&e, 0, sizeof(e));
    e.kp = reinterpret_cast<const KParams*>(c->ws + c->L.consts);
    e.kb = reinterpret_cast<const KBufs*>(c->ws + c->L.consts + align_up(sizeof(KParams), 256));
    e.f[0] = c->f[0];
    e.f[1] = c->f[1];
    e.t0 = c->t;
    e.cur0 = c->cur;
    e.lv = sweep2_args(c, c->t + 1, 2, 1);  // tiling; the levels are set per launch
    b->ch.push_back(c);
    b->gen_expect.push_back(c->gen);
  }
  for (int i = 0; i < n && !B.two; ++i) {
    lbsep_channel* c = chans[i];
    BatchEntry& e = host[i];
    std::memset(&e, 0, sizeof(e));
    e.kp = c->kp;
    e.kb = c->kb;
    e.f[0] = c->f[0];
    e.f[1] = c->f[1];
    e.t0 = c->t;
    e.t_first = c->t_first;
    e.cur0 = c->cur;
    e.split = c->L.split ? 1 : 0;
    if (!c->L.split) node_state += c->L.state_buf;
    b->ch.push_back(c);
    b->gen_expect.push_back(c->gen);
  }
  // non-temporal stores once the one-lane-per-node members' states outgrow
  // half the last-level cache together
  b->nt = node_state > (128ull << 20);
  const long long zero = 0;
  int rc = check_hip(hipMemcpyAsync(b->counter, &zero, sizeof(zero), hipMemcpyHostToDevice, b->stream), "batch copy");
  static const Batch2Levels start{0, 0, 0, 0};
  if (!rc && B.two)
    rc = check_hip(hipMemcpyAsync(b->tab2, host2.data(), n * sizeof(Batch2Entry), hipMemcpyHostToDevice, b->stream),
                   "batch copy");
  if (!rc && B.two)
    rc = check_hip(hipMemcpyAsync(b->lev2, &start, sizeof(start), hipMemcpyHostToDevice, b->stream), "batch copy");
  if (!rc && !B.two)
    rc = check_hip(hipMemcpyAsync(b->tab, host.data(), n * sizeof(BatchEntry), hipMemcpyHostToDevice, b->stream),
                   "batch copy");
  if (!rc)
    rc = check_hip(hipMemcpyAsync(b->blk_ref, blk.data(), blk.size() * sizeof(int2), hipMemcpyHostToDevice,
                                  b->stream),
                   "batch copy");
  if (!rc) rc = check_hip(hipStreamSynchronize(b->stream), "batch copy");
  if (rc) {
    delete b;
    return rc;
  }
  *out = b;
  return LBSEP_OK;
}

int lbsep_batch_step(lbsep_batch* b, int64_t nsteps) {
  if (!b) return fail(LBSEP_EINVAL, "batch is NULL");
  if (nsteps < 0) return fail(LBSEP_EINVAL, "nsteps must be >= 0");
  // the device table holds each member's level and current buffer as of the
  // batch's creation: any change of a member's state since (a step, a set at
  // any level) leaves the table stale
  for (size_t i = 0; i < b->ch.size(); ++i)
    if (b->ch[i]->gen != b->gen_expect[i])
      return fail(LBSEP_EINVAL, "channel " + std::to_string(i) + " was stepped or reset outside its batch");
  int64_t left = nsteps;
  std::vector<int64_t> runs;  // level counts of the graph replays and the eager rest, in order
  while (b->exec && left >= b->graph_steps) {
    if (int e = check_hip(hipGraphLaunch(b->exec, b->stream), "batch graph launch")) return e;
    left -= b->graph_steps;
    runs.push_back(b->graph_steps);
  }
  if (left > 0) {
    enqueue_batch_steps(b, left);
    runs.push_back(left);
  }
  for (size_t i = 0; i < b->ch.size(); ++i) {
    lbsep_channel* c = b->ch[i];
    if (b->two) {
      // the host side of each two-level launch, as in lbsep_step
      for (int64_t run : runs)
        for (int64_t n = run; n > 0;) {
          const int nlev = n >= 2 ? 2 : 1;
          c->pipe2 = true;
          c->glob_next = c->strip_next;
          c->strip_next = c->t + 1;
          c->prev_buf = nlev == 2 ? -1 : c->cur;
          c->cur = 1 - c->cur;
          c->prev_pre = false;
          c->t += nlev;
          c->finalized = false;
          n -= nlev;
        }
    } else {
      c->t += nsteps;
      c->cur = (c->cur + (int)(nsteps & 1)) & 1;
      if (nsteps > 0) {
        c->prev_pre = false;
        c->prev_buf = 1 - c->cur;
        c->finalized = false;
      }
    }
    if (nsteps > 0) ++c->gen;
    b->gen_expect[i] = c->gen;
  }
  return check_hip(hipGetLastError(), "batch step launch");
}

int lbsep_batch_capture(lbsep_batch* b, int64_t steps) {
  if (!b) return fail(LBSEP_EINVAL, "batch is NULL");
  drop_graph(b);
  if (steps <= 0) return LBSEP_OK;
  if (steps > 100000) return fail(LBSEP_EINVAL, "at most 100000 steps per graph");
  if (!b->stream) return fail(LBSEP_EINVAL, "graph capture needs a non-default stream");
  int rc = check_hip(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal), "begin capture");
  if (rc) return rc;
  enqueue_batch_steps(b, steps);
  hipGraph_t g = nullptr;
  rc = check_hip(hipStreamEndCapture(b->stream, &g), "end capture");
  if (rc) return rc;
  hipGraphExec_t x = nullptr;
  rc = check_hip(hipGraphInstantiate(&x, g, nullptr, nullptr, 0), "graph instantiate");
  if (rc) {
    (void)hipGraphDestroy(g);
    return rc;
  }
  b->graph = g;
  b->exec = x;
  b->graph_steps = steps;
  // move the executable graph to the device now rather than on its first replay
  return check_hip(hipGraphUpload(x, b->stream), "graph upload");
}

int32_t lbsep_batch_size(const lbsep_batch* b) { return b ? (int32_t)b->ch.size() : -1; }

void lbsep_batch_destroy(lbsep_batch* b) {
  if (!b) return;
  drop_graph(b);
  delete b;
}

}  // extern "C"
