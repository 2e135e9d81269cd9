// Device code of libvlbm for gfx950 (CDNA4, wave64).
//
// The hot kernel is `step_kernel`: one workgroup per tile of active cells. It
// first executes the tile's interface/boundary tasks (ghost slots read only by
// this tile's own cells, reflux captures), then, after one workgroup barrier,
// advances every cell of the tile: pull the four inbound populations (exact
// shift, paper Sec. 2.2), relax them towards the vectorial equilibrium
// (eqs. num-equilibrium, num-relaxation), and store the 16 post-collision
// values. Populations are stored structure-of-arrays, one plane per (q,k), so
// every load and store of a wavefront is a contiguous run along x.
//
// Arithmetic contract (identical operation order in every implementation, so
// FP64 results are reproducible bit for bit; built with -ffp-contract=off):
//   W_k = ((f_{0k} + f_{1k}) + f_{2k}) + f_{3k}
//   u = m_x / rho; v = m_y / rho; p = (gamma-1) (E - 0.5 (m_x u + m_y v))
//   Q_x = (m_x, m_x u + p, m_y u, (E+p) u);  Q_y = (m_y, m_x v, m_y v + p, (E+p) v)
//   f^eq_{+-x,k} = 0.25 W_k +- h Q_{x,k},  f^eq_{+-y,k} = 0.25 W_k +- h Q_{y,k},  h = 1/(2c)
//   f*_{qk} = f_{qk} + 2beta (f^eq_{qk} - f_{qk})
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include "vlbm_internal.hpp"

namespace vlbm {

// Pressure of the equation of state (EosT); kind is launch-uniform.
template <class T>
__device__ __forceinline__ T pressure(const EosT<T> &e, T rho, T eint) {
  if (e.kind == 1) return e.gm1 * eint - e.ga;
  if (e.kind == 2) {
    const T ar = (e.a * rho) * rho;
    return e.gm1 * (eint + ar) / (T(1) - e.b * rho) - ar;
  }
  return e.gm1 * eint;
}

template <class T>
__device__ __forceinline__ EosT<T> eos_of(const LevelDesc &A) {
  return EosT<T>{A.eos, (T)A.gm1, (T)A.eos_a, (T)A.eos_b, (T)A.eos_ga};
}

template <class T>
__device__ __forceinline__ void relax(T g[16], const EosT<T> &eos, T h, T tb) {
  T W[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) W[k] = ((g[k] + g[4 + k]) + g[8 + k]) + g[12 + k];
  const T rho = W[0], mx = W[1], my = W[2], E = W[3];
  const T u = mx / rho;
  const T v = my / rho;
  const T eint = E - T(0.5) * (mx * u + my * v);
  const T p = pressure<T>(eos, rho, eint);
  const T Qx[4] = {mx, mx * u + p, my * u, (E + p) * u};
  const T Qy[4] = {my, mx * v, my * v + p, (E + p) * v};
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const T w = T(0.25) * W[k];
    const T hx = h * Qx[k];
    const T hy = h * Qy[k];
    g[k] = g[k] + tb * ((w + hx) - g[k]);
    g[4 + k] = g[4 + k] + tb * ((w - hx) - g[4 + k]);
    g[8 + k] = g[8 + k] + tb * ((w + hy) - g[8 + k]);
    g[12 + k] = g[12 + k] + tb * ((w - hy) - g[12 + k]);
  }
}

// Equilibrium of a conserved state, FP64 (inflow ghosts, set_state).
__device__ __forceinline__ void equilibrium(const double W[4], const EosT<double> &eos, double h,
                                            double f[16]) {
  const double rho = W[0], mx = W[1], my = W[2], E = W[3];
  const double u = mx / rho;
  const double v = my / rho;
  const double eint = E - 0.5 * (mx * u + my * v);
  const double p = pressure<double>(eos, rho, eint);
  const double Qx[4] = {mx, mx * u + p, my * u, (E + p) * u};
  const double Qy[4] = {my, mx * v, my * v + p, (E + p) * v};
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const double w = 0.25 * W[k];
    f[k] = w + h * Qx[k];
    f[4 + k] = w - h * Qx[k];
    f[8 + k] = w + h * Qy[k];
    f[12 + k] = w - h * Qy[k];
  }
}

__device__ __forceinline__ double minmod(double a, double b) {
  if (a > 0.0 && b > 0.0) return a < b ? a : b;
  if (a < 0.0 && b < 0.0) return a > b ? a : b;
  return 0.0;
}

// ---------------------------------------------------------------------------
// Interface and boundary tasks (all arithmetic in FP64; stored in T)
// ---------------------------------------------------------------------------
template <class T>
__device__ __forceinline__ void run_task(const LevelDesc &A, int first, double ak, double hd, const Task &t) {
  T *S = static_cast<T *>(A.src);
  const int64_t P = A.plane;
  const int q = t.q;
  const bool book = (t.kind & TASK_LEDGER) != 0;
  switch (t.kind & 0xFF) {
    case T_COPY:
#pragma unroll
      for (int k = 0; k < 4; ++k) S[(q * 4 + k) * P + t.dst] = S[(q * 4 + k) * P + t.src];
      break;
    case T_OUTFLOW:
    case T_REFLECT:
    case T_INFLOW: {
      const int side = t.n0;
      const int qo = q ^ 1;  // opposite population: +x <-> -x, +y <-> -y
      const int kind = t.kind & 0xFF;
      double in[4];
      if (kind == T_OUTFLOW) {
#pragma unroll
        for (int k = 0; k < 4; ++k) in[k] = (double)S[(q * 4 + k) * P + t.src];
      } else if (kind == T_REFLECT) {
        const int kn = side < 2 ? 1 : 2;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const double w = (double)S[(qo * 4 + k) * P + t.src];
          in[k] = (k == kn) ? -w : w;
        }
      } else {
        // constant indices only, so nothing lands in scratch memory
        double W[4], f[16];
#pragma unroll
        for (int k = 0; k < 4; ++k)
          W[k] = side == 0 ? A.win[0][k] : side == 1 ? A.win[1][k] : side == 2 ? A.win[2][k] : A.win[3][k];
        equilibrium(W, eos_of<double>(A), hd, f);
#pragma unroll
        for (int k = 0; k < 4; ++k)
          in[k] = (double)(T)(q == 0 ? f[k] : q == 1 ? f[4 + k] : q == 2 ? f[8 + k] : f[12 + k]);
      }
      double *L = A.ledger + 4 * (int64_t)t.slot;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const T vin = (T)in[k];
        S[(q * 4 + k) * P + t.dst] = vin;
        if (book) {
          const double out = (double)S[(qo * 4 + k) * P + t.src];
          double l = L[k] + A.w2 * (double)vin;
          L[k] = l + (-1.0) * (A.w2 * out);
        }
      }
      break;
    }
    case T_RECON: {
      const T *C = static_cast<const T *>(A.pcur);
      const T *Pv = static_cast<const T *>(A.pprev);
      const int64_t P2 = A.pplane;
      const double bj = (double)(2 * t.j - A.r + 1) / (double)(2 * A.r);
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int64_t pl = (q * 4 + k) * P2;
        const double out = (double)C[pl + t.src];
        const double prev = (double)Pv[pl + t.src];
        double sigma = 0.0;
        if (t.n0 >= 0 && t.n1 >= 0) {
          const double fm = (double)C[pl + t.n0];
          const double fp = (double)C[pl + t.n1];
          sigma = minmod(out - fm, fp - out);
        }
        const double B = out - prev;
        double v = out + B * ak;
        v = v + sigma * bj;
        S[(q * 4 + k) * P + t.dst] = (T)v;
      }
      break;
    }
    case T_REFLUX:
#pragma unroll
      for (int k = 0; k < 4; ++k)
        S[(q * 4 + k) * P + t.dst] = (T)(A.acc_in[4 * (int64_t)t.slot + k] / A.rr);
      break;
    case T_CAPTURE: {
      double *acc = A.acc_out + 4 * (int64_t)t.slot;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        double s = first ? 0.0 : acc[k];
        const int64_t base = (q * 4 + k) * P + t.src;
        for (int j = 0; j < A.r; ++j) s = s + (double)S[base + (int64_t)j * t.n0];
        acc[k] = s;
      }
      break;
    }
    default:
      break;
  }
}

// ---------------------------------------------------------------------------
// The fused step kernel
// ---------------------------------------------------------------------------
// S: storage type of the populations, C: type the relaxation computes in.
// Population planes live in global memory: loads and stores through global
// (not generic) pointers, so no aperture check and no LDS counter in the waits.
template <class S>
using gptr = __attribute__((address_space(1))) S *;

template <class S, class C>
__device__ __forceinline__ void pull(const S *__restrict__ s0, int64_t P, int pitch, int64_t o,
                                     C g[16]) {
  const auto s = (__attribute__((address_space(1))) const S *)s0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    g[k] = (C)s[(0 * 4 + k) * P + o - 1];           // +x arrives from x-1
    g[4 + k] = (C)s[(1 * 4 + k) * P + o + 1];       // -x arrives from x+1
    g[8 + k] = (C)s[(2 * 4 + k) * P + o - pitch];   // +y arrives from y-1
    g[12 + k] = (C)s[(3 * 4 + k) * P + o + pitch];  // -y arrives from y+1
  }
}

template <class S, class C, bool NT>
__device__ __forceinline__ void put(S *__restrict__ d0, int64_t P, int64_t o, const C g[16]) {
  const auto d = (gptr<S>)d0;
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const S v = (S)g[i];
    if (NT)
      __builtin_nontemporal_store(v, &d[i * P + o]);
    else
      d[i * P + o] = v;
  }
}

// Euler flux of a conserved state in FP64 (the order of the arithmetic
// contract above).
__device__ __forceinline__ void euler_flux(const EosT<double> &eos, const double W[4], double Qx[4],
                                           double Qy[4]) {
  const double rho = W[0], mx = W[1], my = W[2], E = W[3];
  const double u = mx / rho;
  const double v = my / rho;
  const double eint = E - 0.5 * (mx * u + my * v);
  const double p = pressure<double>(eos, rho, eint);
  Qx[0] = mx;
  Qx[1] = mx * u + p;
  Qx[2] = my * u;
  Qx[3] = (E + p) * u;
  Qy[0] = my;
  Qy[1] = mx * v;
  Qy[2] = my * v + p;
  Qy[3] = (E + p) * v;
}

// m_k := max(m_k, |Qx_k(W)|, |Qy_k(W)|)
__device__ __forceinline__ void flux_absmax(const EosT<double> &eos, const double W[4], double m[4]) {
  double qx[4], qy[4];
  euler_flux(eos, W, qx, qy);
#pragma unroll
  for (int k = 0; k < 4; ++k) m[k] = fmax(m[k], fmax(fabs(qx[k]), fabs(qy[k])));
}

// Workgroup maximum of m[4] into qmax[4] (bit patterns: non-negative doubles
// order like them, so an unsigned 64-bit atomic max is exact). Every thread of
// the workgroup must call it.
__device__ __forceinline__ void block_qmax(double m[4], unsigned long long *qmax) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1)
#pragma unroll
    for (int k = 0; k < 4; ++k) m[k] = fmax(m[k], __shfl_xor(m[k], off));
  __shared__ double red[4][4];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0)
#pragma unroll
    for (int k = 0; k < 4; ++k) red[k][wv] = m[k];
  __syncthreads();
  if (threadIdx.x < 4) {
    const int k = threadIdx.x;
    double v = red[k][0];
    for (int i = 1; i < (int)(blockDim.x >> 6); ++i) v = fmax(v, red[k][i]);
    const unsigned long long bits = (unsigned long long)__double_as_longlong(v);
    unsigned long long *q = qmax + k;
    // the running maximum only grows: a stale read can only let an update through
    if (bits > __hip_atomic_load(q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) atomicMax(q, bits);
  }
}

// Adaptive time step: the per-cell term of the CFL bound, max over both axes of
// |u_alpha| + c_s, c_s = sqrt(gamma p / rho), from a cell's conserved state.
__device__ __forceinline__ double cfl_term(const EosT<double> &eos, double gamma, const double w[4]) {
  const double u = w[1] / w[0];
  const double v = w[2] / w[0];
  const double p = pressure<double>(eos, w[0], w[3] - 0.5 * (w[1] * u + w[2] * v));
  const double cs = sqrt((gamma * p) / w[0]);
  const double a = fabs(u) + cs, b = fabs(v) + cs;
  return a > b ? a : b;
}

// W of a cell from its stored populations (FP64 sums in the fixed order).
template <class T>
__device__ __forceinline__ void stored_W(const T *s0, int64_t P, int64_t o, double w[4]) {
  const auto s = (__attribute__((address_space(1))) const T *)s0;
#pragma unroll
  for (int k = 0; k < 4; ++k)
    w[k] = (((double)s[(0 * 4 + k) * P + o] + (double)s[(1 * 4 + k) * P + o]) +
            (double)s[(2 * 4 + k) * P + o]) + (double)s[(3 * 4 + k) * P + o];
}

// W of a cell from the populations it is about to store: each rounded to the
// storage type, then summed in FP64 in the fixed order of stored_W below, so
// the value equals what stored_W gives for the stored cell.
template <class T, class C>
__device__ __forceinline__ void W_as_stored(const C g[16], double w[4]) {
#pragma unroll
  for (int k = 0; k < 4; ++k)
    w[k] = (((double)(T)g[k] + (double)(T)g[4 + k]) + (double)(T)g[8 + k]) + (double)(T)g[12 + k];
}

// Fold a workgroup's maximum of non-negative doubles into *slot (as bits,
// which order like the doubles); red: LDS scratch of one double per wave.
// Every thread of the workgroup must call it.
__device__ __forceinline__ void block_max_slot(double m, unsigned long long *slot, double *red) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double v = red[0];
    for (int i = 1; i < (int)(blockDim.x >> 6); ++i) v = fmax(v, red[i]);
    const unsigned long long bits = (unsigned long long)__double_as_longlong(v);
    // the running maximum only grows: a stale read can only let an update through
    if (bits > __hip_atomic_load(slot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) atomicMax(slot, bits);
  }
}

// Offset of level cell (x + dx, y + dy) (active, per its mask bit), periodic
// wrap applied: a neighbour across a periodic x edge sits Nx columns back in
// its row; across a periodic y edge it lies in another stored row, found from
// the frame's row table (the rows next to an active cell are one pitch away).
__device__ __forceinline__ int64_t nb_offset(const LevelDesc &A, int64_t o, int x, int y, int dx, int dy,
                                             int pitch, int Nx, int Ny) {
  int xx = x + dx, yy = y + dy;
  int64_t e = o + dx;
  if (xx < 0) e += Nx, xx += Nx;
  if (xx >= Nx) e -= Nx, xx -= Nx;
  if (yy < 0 || yy >= Ny) {
    yy = yy < 0 ? yy + Ny : yy - Ny;
    return (int64_t)A.srow[yy - A.fy0] * pitch + (xx - A.fx0) + A.xoff;
  }
  return e + (int64_t)dy * pitch;
}

// Level coordinates of a tile's first cell.
__device__ __forceinline__ void tile_origin(const LevelDesc &A, const Tile &tl, int &x0, int &y0) {
  const int rel = tl.off0 - A.xoff;
  const int sr = rel / A.pitch;
  x0 = A.fx0 + (rel - sr * A.pitch);
  y0 = A.fy0 + A.yrow[sr];
}

// The W sets of the adaptive relaxation hold the four components of a cell
// next to each other (element o at 4 o .. 4 o + 3): two 16-byte accesses per
// cell.
typedef double dvec2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void load_W4(const __attribute__((address_space(1))) double *W, int64_t o,
                                        double w[4]) {
  const auto v = (const __attribute__((address_space(1))) dvec2 *)(W + 4 * o);
  const dvec2 a = v[0], b = v[1];
  w[0] = a.x;
  w[1] = a.y;
  w[2] = b.x;
  w[3] = b.y;
}
__device__ __forceinline__ void store_W4(__attribute__((address_space(1))) double *W, int64_t o,
                                         const double w[4]) {
  const auto v = (__attribute__((address_space(1))) dvec2 *)(W + 4 * o);
  v[0] = dvec2{w[0], w[1]};
  v[1] = dvec2{w[2], w[3]};
}

// One workgroup's work on tile `lb` of descriptor A (inlined twice below, so
// that A is either plain kernel-argument memory or plain global memory).
template <class T, class C, bool NT, bool TWO, bool SEN, bool CFL>
__device__ __forceinline__ void run_tile(const LevelDesc &A, int lb, int nblocks, int first,
                                         double ak, int flags) {
  // adaptive time step: this coarse step's h, and the hand-off's dt ratio when
  // the parent last stepped in the previous coarse step
  const bool adt = (flags & STEP_ADAPTIVE_DT) != 0;
  // Tile order. Natural order keeps every workgroup of the chip inside one
  // narrow sweep front (few open DRAM pages); the XCD-contiguous order gives
  // each XCD's L2 a contiguous run of tiles instead.
  const int tid = (flags & STEP_XCD_CONTIGUOUS) ? (lb & 7) * (nblocks >> 3) + (lb >> 3) : lb;
  // Everything the cell loop needs is read before the first store, so it stays
  // in scalar registers (loads after a store may not be scalarised).
  const int ntiles = A.ntiles;
  if (tid >= ntiles) return;
  const Tile tl = A.tiles[tid];
  const T *__restrict__ s = static_cast<const T *>(A.src);
  T *__restrict__ d = static_cast<T *>(A.dst);
  const int64_t plane = A.plane;
  const int pitch = A.pitch;
  const EosT<C> eos = eos_of<C>(A);
  const double hd = adt ? A.dyn[DYN_H] : A.h;
  if (adt && A.use_ratio) ak = ak * (A.dyn[DYN_C_PREV] / A.dyn[DYN_C]);
  const C h = (C)hd, tb = (C)A.tb;
  // adaptive time step: the level's last step of the coarse step folds the
  // CFL term of every cell it stores into the next coarse step's bound (a
  // variant of its own, so that the other launches keep their registers)
  const bool cfl = CFL && adt && A.emit_cfl != 0;
  // adaptive relaxation (eq. sensor-B): per-cell beta out, W of the stored
  // result out, and on a level's last step of the coarse step the next max |Q|
  const auto Sp = (gptr<double>)(SEN ? A.sen : nullptr);
  const auto Wn = (gptr<double>)(SEN ? A.wnext : nullptr);
  const auto M = (__attribute__((address_space(1))) const uint32_t *)(SEN ? A.mask : nullptr);
  const bool emit = SEN && A.emit_qmax != 0;
  const EosT<double> eosd = eos_of<double>(A);
  const double cs = A.c_sensor, bmax = A.beta_max, bspan = A.beta_max - A.beta_min;
  const int Nx = A.Nx, Ny = A.Ny;
  int x0 = 0, y0 = 0;
  if (SEN) tile_origin(A, tl, x0, y0);
  double m[4] = {0.0, 0.0, 0.0, 0.0};
  if (tl.ntask) {
    for (int i = threadIdx.x; i < tl.ntask; i += blockDim.x)
      run_task<T>(A, first, ak, hd, A.tasks[tl.task0 + i]);
    __syncthreads();
  }
  const int n = tl.w * tl.h;
  // the context's first phase clears the next coarse step's Qmax slot when it
  // does not accumulate into it itself (else stage 1 cleared it before)
  if (SEN && A.clear_next && !A.emit_qmax && lb == 0 && threadIdx.x < 4) A.qmax_next[threadIdx.x] = 0ull;
  // Adaptive relaxation (eq. sensor-B) from the W set of the input time level,
  // in LDS: (A) flux and velocity of every active cell within two cells of
  // the tile, each computed once; (B) activity a of the tile and of its
  // one-cell ring and gate theta of the tile, from (A). A cell beyond the tile
  // is reached by at most two mask-checked steps from the nearest tile cell
  // (diagonal first), so only active cells are read and no read leaves the
  // frame; a cell two steps out is used only by the ring cell it is reached
  // through.
  //
  // A tile has at most SEN_TW x SEN_TH <= blockDim.x cells, one per thread.
  // Passes, each ended by a barrier:
  //   0. each thread issues the pull of its cell (kept in registers through
  //      the sensor passes, so that the population loads are in flight while
  //      the sensor runs) and stores its cell's neighbourhood mask in LDS;
  //   1. (A); whether a cell within two of the tile is reached, and through
  //      which ring cell, follows from the nearest tile cell's mask alone
  //      (its bits cover every cell of the walk);
  //   2. (B), from LDS only; the ring cells' neighbours are active or not
  //      per the nearest tile cell's mask as well.
  // Block-sized LDS arrays (tile plus two cells) have the constant stride
  // SEN_TW + 4, ring-sized ones (tile plus one cell) SEN_TW + 2.
  constexpr int RW = SEN_TW + 2, BW = SEN_TW + 4;
  const uint32_t *mt_l = nullptr;  // the tile cells' masks, stride SEN_TW
  double *a_l = nullptr, *th_l = nullptr;
  [[maybe_unused]] C gpre[16];
  if constexpr (SEN) {
    __shared__ double qx_l[4][SEN_BLOCK], qy_l[4][SEN_BLOCK], u_l[SEN_BLOCK], v_l[SEN_BLOCK];
    __shared__ double a_lds[SEN_RING], th_lds[SEN_TW * SEN_TH];
    __shared__ uint32_t mt_lds[SEN_TW * SEN_TH];
    a_l = a_lds;
    th_l = th_lds;
    mt_l = mt_lds;
    const int tw = tl.w, th_ = tl.h;
    // is the cell (dx, dy) away from the tile cell with mask m active?
    auto act = [](uint32_t m, int dx, int dy) -> bool { return (m >> nb_bit(dx, dy)) & 1u; };
    // pass 0
    if ((int)threadIdx.x < n) {
      const int cy = threadIdx.x / tw, cx = threadIdx.x - cy * tw;
      const int64_t o = (int64_t)tl.off0 + (int64_t)cy * pitch + cx;
      pull<T, C>(s, plane, pitch, o, gpre);
      mt_lds[cy * SEN_TW + cx] = M[o];
    }
    __syncthreads();
    // pass 1 (A). Where the tile's block (two cells around it) stays inside
    // the level, no walk wraps and cell (i, j) of the block sits at
    // off0 + j pitch + i (the rows next to an active cell are one pitch away).
    const auto Wc = (__attribute__((address_space(1))) const double *)A.wcur;
    const bool inner = x0 >= 2 && y0 >= 2 && x0 + tw + 2 <= Nx && y0 + th_ + 2 <= Ny;
    for (int p = threadIdx.x; p < SEN_BLOCK; p += blockDim.x) {
      const int bj = p / BW, bi = p - bj * BW;
      const int j = bj - 2, i = bi - 2;
      if (i >= tw + 2 || j >= th_ + 2) continue;
      const int ci = i < 0 ? 0 : i >= tw ? tw - 1 : i, cj = j < 0 ? 0 : j >= th_ ? th_ - 1 : j;
      const int di = i - ci, dj = j - cj;
      if ((di == 2 || di == -2) && (dj == 2 || dj == -2)) continue;  // block corners: never used
      const int sx = (di > 0) - (di < 0), sy = (dj > 0) - (dj < 0);
      // first step to the tile or ring cell (ci + sx, cj + sy), then on to
      // (ci + di, cj + dj): both cells active
      const uint32_t mt = mt_lds[cj * SEN_TW + ci];
      if (!act(mt, sx, sy) || !act(mt, di, dj)) continue;
      int64_t o;
      if (inner) {
        o = (int64_t)tl.off0 + (int64_t)j * pitch + i;
      } else {
        o = (int64_t)tl.off0 + (int64_t)cj * pitch + ci;
        int x = x0 + ci, y = y0 + cj;
        if (sx != 0 || sy != 0) {
          o = nb_offset(A, o, x, y, sx, sy, pitch, Nx, Ny);
          x += sx;
          y += sy;
          x = x < 0 ? x + Nx : x >= Nx ? x - Nx : x;
          y = y < 0 ? y + Ny : y >= Ny ? y - Ny : y;
        }
        if (di != sx || dj != sy) o = nb_offset(A, o, x, y, di - sx, dj - sy, pitch, Nx, Ny);
      }
      double w[4], qx[4], qy[4];
      load_W4(Wc, o, w);
      euler_flux(eosd, w, qx, qy);
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        qx_l[k][p] = qx[k];
        qy_l[k][p] = qy[k];
      }
      u_l[p] = w[1] / w[0];
      v_l[p] = w[2] / w[0];
    }
    __syncthreads();
    // pass 2 (B)
    double qm[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) qm[k] = __longlong_as_double((long long)A.qmax[k]);
    for (int p = threadIdx.x; p < SEN_RING; p += blockDim.x) {
      const int rj = p / RW, ri = p - rj * RW;
      if (ri >= tw + 2 || rj >= th_ + 2) continue;
      const int i = ri - 1, j = rj - 1;
      const int ci = i < 0 ? 0 : i >= tw ? tw - 1 : i, cj = j < 0 ? 0 : j >= th_ ? th_ - 1 : j;
      const int ai = i - ci, aj = j - cj;  // this cell relative to the nearest tile cell
      const uint32_t mt = mt_lds[cj * SEN_TW + ci];
      double a = 0.0, th = 0.0;
      if (act(mt, ai, aj)) {
        // s_k from the four neighbours' fluxes over this coarse step's Qmax,
        // a their RMS; theta from dilatation and vorticity. A neighbour that
        // is not an active cell stands in as the cell itself.
        const int pb = (j + 2) * BW + i + 2;
        constexpr int DX[4] = {1, -1, 0, 0}, DY[4] = {0, 0, 1, -1};
        int e[4];
#pragma unroll
        for (int d = 0; d < 4; ++d) e[d] = act(mt, ai + DX[d], aj + DY[d]) ? pb + DX[d] + DY[d] * BW : pb;
        double sk[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const double dq = (qx_l[k][e[0]] - qx_l[k][e[1]]) + (qy_l[k][e[2]] - qy_l[k][e[3]]);
          sk[k] = qm[k] > 0.0 ? (0.5 * dq) / qm[k] : 0.0;
        }
        a = sqrt(0.25 * (((sk[0] * sk[0] + sk[1] * sk[1]) + sk[2] * sk[2]) + sk[3] * sk[3]));
        const double dil = 0.5 * ((u_l[e[0]] - u_l[e[1]]) + (v_l[e[2]] - v_l[e[3]]));
        const double vort = 0.5 * ((v_l[e[0]] - v_l[e[1]]) - (u_l[e[2]] - u_l[e[3]]));
        const double den = dil * dil + vort * vort;
        th = (dil < 0.0 && den > 0.0) ? (dil * dil) / den : 0.0;
      }
      a_l[p] = a;
      if (i >= 0 && i < tw && j >= 0 && j < th_) th_l[j * SEN_TW + i] = th;
    }
    __syncthreads();
  }
  // with cfl, the CFL term of every stored cell (from the values as stored)
  // joins the next coarse step's bound
  double mc = 0.0;
  double gam = 0.0;
  EosT<double> eosc{};
  if (cfl) {
    eosc = eos_of<double>(A);
    gam = A.dyn[DYN_GAMMA];
  }
  if (TWO && !SEN) {
    // two cells per thread, both gathers issued before either relaxation
    for (int c = threadIdx.x; c < n; c += 2 * blockDim.x) {
      const int c2 = c + blockDim.x;
      const int cy = c / tl.w, cx = c - cy * tl.w;
      const int64_t o = (int64_t)tl.off0 + (int64_t)cy * pitch + cx;
      C g[16], g2[16];
      pull<T, C>(s, plane, pitch, o, g);
      int64_t o2 = 0;
      if (c2 < n) {
        const int cy2 = c2 / tl.w, cx2 = c2 - cy2 * tl.w;
        o2 = (int64_t)tl.off0 + (int64_t)cy2 * pitch + cx2;
        pull<T, C>(s, plane, pitch, o2, g2);
      }
      relax<C>(g, eos, h, tb);
      put<T, C, NT>(d, plane, o, g);
      if (cfl) {
        double w[4];
        W_as_stored<T, C>(g, w);
        mc = fmax(mc, cfl_term(eosc, gam, w));
      }
      if (c2 < n) {
        relax<C>(g2, eos, h, tb);
        put<T, C, NT>(d, plane, o2, g2);
        if (cfl) {
          double w[4];
          W_as_stored<T, C>(g2, w);
          mc = fmax(mc, cfl_term(eosc, gam, w));
        }
      }
    }
  } else {
    for (int c = threadIdx.x; c < n; c += blockDim.x) {
      const int cy = c / tl.w;
      const int cx = c - cy * tl.w;
      const int64_t o = (int64_t)tl.off0 + (int64_t)cy * pitch + cx;
      C g[16];
      if (SEN && c == (int)threadIdx.x) {
#pragma unroll
        for (int q = 0; q < 16; ++q) g[q] = gpre[q];
      } else {
        pull<T, C>(s, plane, pitch, o, g);
      }
      C tbc = tb;
      if (SEN) {
        // beta = beta_max - (beta_max - beta_min) clip(C sbar theta, 0, 1),
        // sbar the mean of a over the active cells of the 3 x 3 block, summed
        // row by row from (x - 1, y - 1)
        const int pc = (cy + 1) * RW + cx + 1;
        const uint32_t mk = mt_l[cy * SEN_TW + cx];
        double sum = 0.0;
        int cnt = 0;
#pragma unroll
        for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
          for (int dx = -1; dx <= 1; ++dx) {
            if ((mk >> nb_bit(dx, dy)) & 1) {
              sum += a_l[pc + dy * RW + dx];
              ++cnt;
            }
          }
        double z = (cs * (sum / (double)cnt)) * th_l[cy * SEN_TW + cx];
        z = z < 0.0 ? 0.0 : z > 1.0 ? 1.0 : z;
        const double beta = bmax - bspan * z;
        if (emit) Sp[SEN_BETA * plane + o] = beta;  // beta of the level's last step of the coarse step
        tbc = (C)(2.0 * beta);
      }
      relax<C>(g, eos, h, tbc);
      put<T, C, NT>(d, plane, o, g);
      if (SEN || cfl) {
        double w[4];
        W_as_stored<T, C>(g, w);
        if (SEN) {
          store_W4(Wn, o, w);
          if (emit) flux_absmax(eosd, w, m);
        }
        if (cfl) mc = fmax(mc, cfl_term(eosc, gam, w));
      }
    }
  }
  if (emit) block_qmax(m, A.qmax_next);
  if (cfl) {
    __shared__ double red[16];
    block_max_slot(mc, A.cfl_next, red);
  }
}

// DP_, FB_, NB_ := the descriptor of workgroup b of launch Lc, its
// segment's first workgroup and workgroup count (uniform scalar binary search
// of the segment table). A macro, not a function: through a call the compiler
// loses the descriptor's address space and reads it with vector loads.
#define VLBM_FIND_SEGMENT(LC_, B_, DP_, FB_, NB_)                          \
  const LevelDesc *DP_ = (LC_).d0;                                         \
  int FB_ = 0, NB_ = (LC_).nblocks;                                        \
  if ((LC_).nseg > 0) {                                                    \
    int lo_ = 0, hi_ = (LC_).nseg - 1;                                     \
    while (lo_ < hi_) {                                                    \
      const int mid_ = (lo_ + hi_ + 1) >> 1;                               \
      if ((LC_).segs[mid_].first_block <= (B_)) lo_ = mid_; else hi_ = mid_ - 1; \
    }                                                                      \
    const Segment sg_ = (LC_).segs[lo_];                                   \
    DP_ = sg_.d;                                                           \
    FB_ = sg_.first_block;                                                 \
    NB_ = sg_.nblocks;                                                     \
  }


template <class T, class C, bool NT, bool TWO, bool SEN, bool CFL>
__global__ __launch_bounds__(256) void step_kernel(StepLaunch Lc) {
  const int b = blockIdx.x;
  VLBM_FIND_SEGMENT(Lc, b, dp, first_block, nblocks)
  run_tile<T, C, NT, TWO, SEN, CFL>(*dp, b - first_block, nblocks, Lc.first, Lc.ak, Lc.flags);
}

// ---------------------------------------------------------------------------
// Fused two-sub-step launch of the finest level (r = 2). One workgroup per
// tile of at most FUSE_W x FUSE_H cells, aligned to the 2 x 2 blocks of
// parent cells (so both cells of every reflux capture lie in one tile):
//   1. sub-step-1 ghost values of the tile's cells and of the sources of its
//      ring go into the global ghost slots (neighbouring tiles write the same
//      values);
//   2. sub-step 1 of the tile cells (all populations) and of the active ring
//      cells (the one population the tile pulls from each), rounded to the
//      storage type, into LDS;
//   3. sub-step-2 ghost values into the LDS ring positions, and the parent's
//      reflux accumulators receive both sub-steps' outgoing values;
//   4. sub-step 2 of the tile, pulled from LDS, stored to the next buffer.
// The arithmetic and its rounding points are those of two separate launches,
// so results are bit-identical; the intermediate level never travels to HBM.
// ---------------------------------------------------------------------------
template <class T>
__device__ __forceinline__ void run_task_k2(const LevelDesc &A, double ak2, double hd, const Task &t, T *F1) {
  constexpr int np = FUSE_POS;
  const int q = t.q;
  const int kind = t.kind & 0xFF;
  if (kind == T_RECON) {
    const T *C = static_cast<const T *>(A.pcur);
    const T *Pv = static_cast<const T *>(A.pprev);
    const int64_t P2 = A.pplane;
    const double bj = (double)(2 * t.j - A.r + 1) / (double)(2 * A.r);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int64_t pl = (q * 4 + k) * P2;
      const double out = (double)C[pl + t.src];
      const double prev = (double)Pv[pl + t.src];
      double sigma = 0.0;
      if (t.n0 >= 0 && t.n1 >= 0) sigma = minmod(out - (double)C[pl + t.n0], (double)C[pl + t.n1] - out);
      const double B = out - prev;
      double v = out + B * ak2;
      v = v + sigma * bj;
      F1[(q * 4 + k) * np + t.dst] = (T)v;
    }
    return;
  }
  // boundary kinds: the source is the tile cell's own sub-step-1 value in LDS
  const int side = t.n0;
  const int qo = q ^ 1;
  double in[4];
  if (kind == T_OUTFLOW) {
#pragma unroll
    for (int k = 0; k < 4; ++k) in[k] = (double)F1[(q * 4 + k) * np + t.src];
  } else if (kind == T_REFLECT) {
    const int kn = side < 2 ? 1 : 2;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const double w = (double)F1[(qo * 4 + k) * np + t.n1];
      in[k] = (k == kn) ? -w : w;
    }
  } else {
    double W[4], f[16];
#pragma unroll
    for (int k = 0; k < 4; ++k)
      W[k] = side == 0 ? A.win[0][k] : side == 1 ? A.win[1][k] : side == 2 ? A.win[2][k] : A.win[3][k];
    equilibrium(W, eos_of<double>(A), hd, f);
#pragma unroll
    for (int k = 0; k < 4; ++k)
      in[k] = (double)(T)(q == 0 ? f[k] : q == 1 ? f[4 + k] : q == 2 ? f[8 + k] : f[12 + k]);
  }
  double *L = A.ledger + 4 * (int64_t)t.slot;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const T vin = (T)in[k];
    F1[(q * 4 + k) * np + t.dst] = vin;
    const double out = (double)F1[(qo * 4 + k) * np + t.n1];
    double l = L[k] + A.w2 * (double)vin;
    L[k] = l + (-1.0) * (A.w2 * out);
  }
}

template <class T, class C, bool NT>
__device__ __forceinline__ void fused_tile(const LevelDesc &A, int lb, int nblocks, int flags) {
  constexpr int np = FUSE_POS;
  __shared__ __attribute__((aligned(16))) T F1[16 * FUSE_POS];
  // XCD-contiguous order: a tile's ring cells belong to its neighbours, whose
  // lines then sit in the same XCD's L2
  const int tid = (flags & STEP_XCD_CONTIGUOUS) ? (lb & 7) * (nblocks >> 3) + (lb >> 3) : lb;
  const int ntiles = A.ntiles;
  if (tid >= ntiles) return;
  const Tile tl = A.tiles[tid];
  const T *__restrict__ s = static_cast<const T *>(A.src);
  T *__restrict__ d = static_cast<T *>(A.dst);
  const int64_t plane = A.plane;
  const int pitch = A.pitch;
  const EosT<C> eos = eos_of<C>(A);
  const bool adt = (flags & STEP_ADAPTIVE_DT) != 0;
  const double hd = adt ? A.dyn[DYN_H] : A.h;
  const C h = (C)hd, tb = (C)A.tb;
  const int w = tl.w, w1 = w + 1;
  double ak1 = (double)(1 - A.r) / (double)(2 * A.r);   // k = 1
  double ak2 = (double)(3 - A.r) / (double)(2 * A.r);   // k = 2
  if (adt && A.use_ratio) {
    const double ratio = A.dyn[DYN_C_PREV] / A.dyn[DYN_C];
    ak1 = ak1 * ratio;
    ak2 = ak2 * ratio;
  }
  // adaptive time step: sub-step 2 folds the CFL term of every cell it stores
  // into the next coarse step's bound when this is the level's last launch
  const bool cfl = adt && A.emit_cfl != 0;
  const Task *tk = A.tasks + tl.task0;
  // Items of step 2: the tile cells, then the ring cells. A thread takes item
  // t and item t + blockDim (there are at most FUSE_W x FUSE_H + 2 (FUSE_W +
  // FUSE_H) items); the ring entries are read here, ahead of the first
  // barrier, so the gathers of step 2 wait on nothing but themselves.
  const int ncell = w * tl.h;
  const Task *ring = tk + tl.ntask;
  const int nitem = ncell + tl.nring;
  const int i0 = threadIdx.x, i1 = threadIdx.x + blockDim.x;
  // a thread without an item gathers around the tile's first cell (in bounds:
  // every active cell has its four neighbour slots) and discards the values,
  // so that the gathers are unconditional and the first relaxation waits only
  // for its own sixteen loads
  int64_t src0 = tl.off0, src1 = tl.off0;
  int rq0 = -1, rq1 = -1, rd0 = 0, rd1 = 0;  // ring item: population and LDS position
  if (i0 < ncell) {
    const int cy = i0 / w, cx = i0 - cy * w;
    src0 = (int64_t)tl.off0 + (int64_t)cy * pitch + cx;
  } else if (i0 < nitem) {
    const Task &t = ring[i0 - ncell];
    src0 = t.src;
    rq0 = t.q;
    rd0 = t.dst;
  }
  if (i1 < ncell) {
    const int cy = i1 / w, cx = i1 - cy * w;
    src1 = (int64_t)tl.off0 + (int64_t)cy * pitch + cx;
  } else if (i1 < nitem) {
    const Task &t = ring[i1 - ncell];
    src1 = t.src;
    rq1 = t.q;
    rd1 = t.dst;
  }
  // 1. sub-step-1 ghost values (global)
  for (int i = threadIdx.x; i < tl.ntask; i += blockDim.x) run_task<T>(A, 1, ak1, hd, tk[i]);
  __syncthreads();
  // 2. sub-step 1 of tile and ring cells into LDS: both gathers of a thread
  // are issued before either relaxation, so the ring's round trip overlaps the
  // tile's
  auto item_store = [&](int i, int rq, int rd, const C g[16]) {
    if (rq < 0) {
      const int cy = i / w, cx = i - cy * w;
      const int p0 = cy * w1 + cx + 1, p1 = cy * w1 + cx, p2 = (cy + 1) * w + cx, p3 = cy * w + cx;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        F1[k * np + p0] = (T)g[k];
        F1[(4 + k) * np + p1] = (T)g[4 + k];
        F1[(8 + k) * np + p2] = (T)g[8 + k];
        F1[(12 + k) * np + p3] = (T)g[12 + k];
      }
    } else {
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const C v = rq == 0 ? g[k] : rq == 1 ? g[4 + k] : rq == 2 ? g[8 + k] : g[12 + k];
        F1[(rq * 4 + k) * np + rd] = (T)v;
      }
    }
  };
  {
    const bool has0 = i0 < nitem, has1 = i1 < nitem;
    C g0[16], g1[16];
    pull<T, C>(s, plane, pitch, src0, g0);
    pull<T, C>(s, plane, pitch, src1, g1);
    if (has0) {
      relax<C>(g0, eos, h, tb);
      item_store(i0, rq0, rd0, g0);
    }
    if (has1) {
      relax<C>(g1, eos, h, tb);
      item_store(i1, rq1, rd1, g1);
    }
  }
  __syncthreads();
  // 3. sub-step-2 ghost values into LDS; both sub-steps' reflux captures
  const Task *k2 = ring + tl.nring;
  const Task *cap = k2 + tl.nk2;
  for (int i = threadIdx.x; i < tl.nk2 + tl.ncap; i += blockDim.x) {
    if (i < tl.nk2) {
      run_task_k2<T>(A, ak2, hd, k2[i], F1);
    } else {
      const Task &t = cap[i - tl.nk2];
      double *acc = A.acc_out + 4 * (int64_t)t.slot;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int pl = t.q * 4 + k;
        double v = 0.0;
        for (int j = 0; j < A.r; ++j) v = v + (double)s[pl * plane + t.src + (int64_t)j * t.n0];
        for (int j = 0; j < A.r; ++j) v = v + (double)F1[pl * np + t.n1 + j * t.j];
        acc[k] = v;
      }
    }
  }
  __syncthreads();
  // 4. sub-step 2 of the tile from LDS; with cfl, the CFL term of every
  // stored cell (from the values as stored) joins the next coarse step's bound
  double mc = 0.0;
  double gam = 0.0;
  EosT<double> eosd{};
  if (cfl) {
    eosd = eos_of<double>(A);
    gam = A.dyn[DYN_GAMMA];
  }
  for (int i = threadIdx.x; i < ncell; i += blockDim.x) {
    const int cy = i / w, cx = i - cy * w;
    const int p0 = cy * w1 + cx, p1 = cy * w1 + cx + 1, p2 = cy * w + cx, p3 = (cy + 1) * w + cx;
    C g[16];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      g[k] = (C)F1[k * np + p0];
      g[4 + k] = (C)F1[(4 + k) * np + p1];
      g[8 + k] = (C)F1[(8 + k) * np + p2];
      g[12 + k] = (C)F1[(12 + k) * np + p3];
    }
    relax<C>(g, eos, h, tb);
    const int64_t o = (int64_t)tl.off0 + (int64_t)cy * pitch + cx;
    put<T, C, NT>(d, plane, o, g);
    if (cfl) {
      double wv[4];
      W_as_stored<T, C>(g, wv);
      mc = fmax(mc, cfl_term(eosd, gam, wv));
    }
  }
  if (cfl) {
    __syncthreads();  // every thread is done with F1: the reduction reuses it
    block_max_slot(mc, A.cfl_next, reinterpret_cast<double *>(F1));
  }
}

template <class T, class C, bool NT>
__global__ __launch_bounds__(FUSE_THREADS) void fused_kernel(StepLaunch Lc) {
  const int b = blockIdx.x;
  VLBM_FIND_SEGMENT(Lc, b, dp, first_block, nblocks)
  fused_tile<T, C, NT>(*dp, b - first_block, nblocks, Lc.flags);
}

// ev0/ev1 (may be null): events that take the kernel's own start and end
// times (AMD launch extension), for per-kernel timing without stream markers.
hipError_t launch_step(const StepLaunch &a, int fp32, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
  if (a.nblocks <= 0 || a.nseg < 0) return hipSuccess;
  dim3 grid(a.nblocks), block(256);
  const bool nt = (a.flags & STEP_NT_STORES) != 0, two = (a.flags & STEP_TWO_CELLS) != 0;
  if (a.flags & STEP_FUSED_PHASE) {
    block = dim3(FUSE_THREADS);
#define VLBM_FUSED(S, C)                                                                          \
  do {                                                                                            \
    if (nt) hipExtLaunchKernelGGL((fused_kernel<S, C, true>), grid, block, 0, s, ev0, ev1, 0, a);  \
    else hipExtLaunchKernelGGL((fused_kernel<S, C, false>), grid, block, 0, s, ev0, ev1, 0, a);    \
  } while (0)
    if (!fp32)
      VLBM_FUSED(double, double);
    else if (a.flags & STEP_F64_MATH)
      VLBM_FUSED(float, double);
    else
      VLBM_FUSED(float, float);
#undef VLBM_FUSED
    return hipGetLastError();
  }
  const bool sen = (a.flags & STEP_SENSOR) != 0;  // per-cell beta: one cell per thread
  const bool cfl = (a.flags & STEP_CFL_EMIT) != 0;
#define VLBM_STEP1(S, C, CF)                                                                                \
  do {                                                                                                      \
    if (sen && nt)                                                                                          \
      hipExtLaunchKernelGGL((step_kernel<S, C, true, false, true, CF>), grid, block, 0, s, ev0, ev1, 0, a);   \
    else if (sen)                                                                                           \
      hipExtLaunchKernelGGL((step_kernel<S, C, false, false, true, CF>), grid, block, 0, s, ev0, ev1, 0, a);  \
    else if (nt && two)                                                                                     \
      hipExtLaunchKernelGGL((step_kernel<S, C, true, true, false, CF>), grid, block, 0, s, ev0, ev1, 0, a);   \
    else if (nt)                                                                                            \
      hipExtLaunchKernelGGL((step_kernel<S, C, true, false, false, CF>), grid, block, 0, s, ev0, ev1, 0, a);  \
    else if (two)                                                                                           \
      hipExtLaunchKernelGGL((step_kernel<S, C, false, true, false, CF>), grid, block, 0, s, ev0, ev1, 0, a);  \
    else                                                                                                    \
      hipExtLaunchKernelGGL((step_kernel<S, C, false, false, false, CF>), grid, block, 0, s, ev0, ev1, 0, a); \
  } while (0)
#define VLBM_STEP(S, C)           \
  do {                            \
    if (cfl)                      \
      VLBM_STEP1(S, C, true);     \
    else                          \
      VLBM_STEP1(S, C, false);    \
  } while (0)
  if (!fp32)
    VLBM_STEP(double, double);
  else if (a.flags & STEP_F64_MATH)
    VLBM_STEP(float, double);
  else
    VLBM_STEP(float, float);
#undef VLBM_STEP1
#undef VLBM_STEP
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Space/time-adaptive relaxation parameter (Sec. 2.2, eq. sensor-B) of every
// active cell of a level, from the state at the start of its step, FP64 for
// every storage type:
//   Qmax_k = max over both directions and the active cells of every level of
//      |Q_{alpha,k}(W)|, taken at the start of each coarse step (the one
//      instant at which the whole hierarchy holds one time level);
//   s_k = (0.5 ((Qx_k(x+1) - Qx_k(x-1)) + (Qy_k(y+1) - Qy_k(y-1)))) / Qmax_k
//      (0 where Qmax_k = 0), a = sqrt(0.25 (((s_0^2 + s_1^2) + s_2^2) + s_3^2));
//   dil = 0.5 ((u(x+1) - u(x-1)) + (v(y+1) - v(y-1))),
//   vort = 0.5 ((v(x+1) - v(x-1)) - (u(y+1) - u(y-1))),
//   theta = dil^2 / (dil^2 + vort^2) under compression (dil < 0), else 0
//      (0 too where dil^2 + vort^2 underflows to 0);
//   beta = beta_max - (beta_max - beta_min) clip(C sbar theta, 0, 1), sbar the
//      mean of a over the active cells of the 3 x 3 block (summed row by row
//      from (x - 1, y - 1)).
// A neighbour that is not an active cell of the level (across a non-periodic
// side, outside the frame, a hole, uncovered) stands in as the cell itself in
// the differences and is left out of the mean.
//
// Pipeline. The step kernel (SEN variant) computes, per tile and in LDS, the
// fluxes of the cells within two cells of the tile, a of the tile and its
// ring and theta of the tile, all from the W set of its input time level;
// takes beta of every cell from them, writes beta to its plane, relaxes with
// it, writes W of every cell it advances (the sums of the values it stores)
// into the other W set, and on a level's last step of a coarse step
// accumulates the next coarse step's Qmax from them. The two W sets alternate
// with the level's step count, so no workgroup reads W that another one of
// the same launch writes. (Summing W from the stored populations of the
// block instead, which saves the two W sets' traffic, was measured slower:
// four times the loads per block cell.) The context's first launch of a
// coarse step clears the next Qmax slot (workgroup 0), or stage 1 does just
// before it when that launch also accumulates into the slot; stage 0 fills
// the input W set of every level and this coarse step's Qmax from the stored
// populations, once after any change of state.
// ---------------------------------------------------------------------------

template <class T>
__global__ __launch_bounds__(256) void sensor0_kernel(StepLaunch Lc) {
  VLBM_FIND_SEGMENT(Lc, (int)blockIdx.x, dp, fb, nb)
  (void)nb;
  const LevelDesc &A = *dp;
  const int tid = blockIdx.x - fb;
  if (tid >= A.ntiles || !A.sen) return;  // uniform over the workgroup
  const Tile tl = A.tiles[tid];
  const T *s = static_cast<const T *>(A.src);
  // the W set this descriptor's step reads: the level's current time level
  const auto Wp = (gptr<double>)const_cast<double *>(A.wcur);
  const int64_t P = A.plane;
  const int pitch = A.pitch;
  const EosT<double> eos = eos_of<double>(A);
  double m[4] = {0.0, 0.0, 0.0, 0.0};
  const int n = tl.w * tl.h;
  for (int c = threadIdx.x; c < n; c += blockDim.x) {
    const int cy = c / tl.w, cx = c - cy * tl.w;
    const int64_t o = (int64_t)tl.off0 + (int64_t)cy * pitch + cx;
    double w[4];
    stored_W<T>(s, P, o, w);
    store_W4(Wp, o, w);
    flux_absmax(eos, w, m);
  }
  block_qmax(m, A.qmax);
}

// Stage 1: clear the next coarse step's max |Q| slot of every descriptor of
// the launch that is its context's first phase and also accumulates into
// that slot (a level with one step per coarse step); the step kernel clears
// it for every other first phase. The slot is the one the previous coarse
// step read as its Qmax.
__global__ __launch_bounds__(64) void sensor_clear_kernel(StepLaunch Lc) {
  const int ns = Lc.nseg > 0 ? Lc.nseg : 1;
  for (int i = threadIdx.x; i < 4 * ns; i += blockDim.x) {
    const LevelDesc *D = Lc.nseg > 0 ? Lc.segs[i >> 2].d : Lc.d0;
    if (D->sen && D->clear_next && D->emit_qmax) D->qmax_next[i & 3] = 0ull;
  }
}

// One thread per stored frame element; writes the mask of every active cell
// and 0 elsewhere.
__global__ __launch_bounds__(256) void sensor_mask_kernel(const uint8_t *status, uint32_t *mask,
                                                          const int32_t *srow, const int32_t *yrow, int fx0,
                                                          int fy0, int fw, int fh, int nrows, int pitch,
                                                          int xoff, int Nx, int Ny, int per) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)fw * nrows) return;
  const int sr = (int)(i / fw), fx = (int)(i - (int64_t)sr * fw);
  const int64_t o = (int64_t)sr * pitch + fx + xoff;
  uint32_t mk = 0;
  if (status[i] == 1) {
    const int x = fx0 + fx, y = fy0 + yrow[sr];
    for (int dy = -2; dy <= 2; ++dy)
      for (int dx = -2; dx <= 2; ++dx) {
        if ((dx == 2 || dx == -2) && (dy == 2 || dy == -2)) continue;  // corners: unused
        const int bit = nb_bit(dx, dy);
        int xx = x + dx, yy = y + dy;
        if (xx < 0 || xx >= Nx) {
          if (!(per & 1)) continue;
          xx = ((xx % Nx) + Nx) % Nx;
        }
        if (yy < 0 || yy >= Ny) {
          if (!(per & 2)) continue;
          yy = ((yy % Ny) + Ny) % Ny;
        }
        const int gx = xx - fx0, gy = yy - fy0;
        if (gx < 0 || gy < 0 || gx >= fw || gy >= fh || srow[gy] < 0) continue;
        if (status[(int64_t)srow[gy] * fw + gx] == 1) mk |= 1u << bit;
      }
  }
  mask[o] = mk;
}

hipError_t launch_sensor_mask(const uint8_t *status, uint32_t *mask, const int32_t *srow, const int32_t *yrow,
                              int fx0, int fy0, int fw, int fh, int nrows, int pitch, int xoff, int Nx,
                              int Ny, int per, hipStream_t s) {
  const int64_t n = (int64_t)fw * nrows;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(sensor_mask_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, status, mask,
                     srow, yrow, fx0, fy0, fw, fh, nrows, pitch, xoff, Nx, Ny, per);
  return hipGetLastError();
}

hipError_t launch_sensor(const StepLaunch &a, int stage, int fp32, hipStream_t s) {
  if (a.nblocks <= 0 || a.nseg < 0) return hipSuccess;
  const dim3 grid(a.nblocks), block(256);
  if (stage == 0) {
    if (fp32)
      hipLaunchKernelGGL(sensor0_kernel<float>, grid, block, 0, s, a);
    else
      hipLaunchKernelGGL(sensor0_kernel<double>, grid, block, 0, s, a);
  } else if (stage == 1) {
    hipLaunchKernelGGL(sensor_clear_kernel, dim3(1), dim3(64), 0, s, a);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Adaptive time step: c_n = (kappa D) max over the active cells of every level
// and both axes of |u_alpha| + c_s, c_s = sqrt(gamma p / rho), from the stored
// state at the start of the coarse step; then c_prev := c, c := c_n,
// h := 1 / (2 c_n), t := t + dx0 / c_n (the one-thread finalize), and the max
// slot is cleared for the next coarse step. cfl_kernel takes the bound from
// memory after the host changed the state; otherwise each level's last step
// launch of the previous coarse step has already folded it in (emit_cfl).
// ---------------------------------------------------------------------------
template <class T>
__global__ __launch_bounds__(256) void cfl_kernel(StepLaunch Lc, unsigned long long *cmax, const double *dyn) {
  VLBM_FIND_SEGMENT(Lc, (int)blockIdx.x, dp, fb, nb)
  (void)nb;
  const LevelDesc &A = *dp;
  const int tid = blockIdx.x - fb;
  if (tid >= A.ntiles) return;  // uniform over the workgroup
  const Tile tl = A.tiles[tid];
  const int64_t P = A.plane;
  const int pitch = A.pitch;
  const EosT<double> eos = eos_of<double>(A);
  const double gamma = dyn[DYN_GAMMA];
  double m = 0.0;
  const int n = tl.w * tl.h;
  for (int c = threadIdx.x; c < n; c += blockDim.x) {
    const int cy = c / tl.w, cx = c - cy * tl.w;
    const int64_t o = (int64_t)tl.off0 + (int64_t)cy * pitch + cx;
    double w[4];
    stored_W<T>(static_cast<const T *>(A.src), P, o, w);
    m = fmax(m, cfl_term(eos, gamma, w));
  }
  __shared__ double red[16];
  block_max_slot(m, cmax, red);
}

__global__ void cfl_finalize_kernel(double *dyn, unsigned long long *cmax) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const double m = __longlong_as_double((long long)*cmax);
  const double c = dyn[DYN_KD] * m;
  dyn[DYN_C_PREV] = dyn[DYN_C];
  dyn[DYN_C] = c;
  dyn[DYN_H] = 1.0 / (2.0 * c);
  dyn[DYN_TIME] = dyn[DYN_TIME] + dyn[DYN_DX0] / c;
  *cmax = 0ull;
}

hipError_t launch_cfl(const StepLaunch &a, int fp32, unsigned long long *cmax, const double *dyn,
                      hipStream_t s) {
  if (a.nblocks <= 0 || a.nseg < 0) return hipSuccess;
  const dim3 grid(a.nblocks), block(256);
  if (fp32)
    hipLaunchKernelGGL(cfl_kernel<float>, grid, block, 0, s, a, cmax, dyn);
  else
    hipLaunchKernelGGL(cfl_kernel<double>, grid, block, 0, s, a, cmax, dyn);
  return hipGetLastError();
}

// Zero n 64-bit words: a kernel rather than a memset, because advance may run
// under a caller's stream capture, and a captured memset node is avoided.
__global__ void clear_u64_kernel(unsigned long long *p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0ull;
}

hipError_t launch_clear_u64(unsigned long long *p, int n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(clear_u64_kernel, dim3((n + 63) / 64), dim3(64), 0, s, p, n);
  return hipGetLastError();
}

hipError_t launch_cfl_finalize(double *dyn, unsigned long long *cmax, hipStream_t s) {
  hipLaunchKernelGGL(cfl_finalize_kernel, dim3(1), dim3(64), 0, s, dyn, cmax);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Conservation audit: per-tile compensated sums of sum_q f_{q,k}
// ---------------------------------------------------------------------------
__device__ __forceinline__ void neumaier(double &s, double &c, double v) {
  const double t = s + v;
  if (fabs(s) >= fabs(v))
    c += (s - t) + v;
  else
    c += (v - t) + s;
  s = t;
}

template <class T>
__global__ __launch_bounds__(256) void audit_kernel(const T *__restrict__ buf,
                                                    const Tile *tiles, int64_t P, int pitch,
                                                    double *partial) {
  __shared__ double red[4][256];
  const Tile tl = tiles[blockIdx.x];
  double s[4] = {0, 0, 0, 0}, cc[4] = {0, 0, 0, 0};
  const int n = tl.w * tl.h;
  for (int c = threadIdx.x; c < n; c += blockDim.x) {
    const int cy = c / tl.w;
    const int cx = c - cy * tl.w;
    const int64_t o = (int64_t)tl.off0 + (int64_t)cy * pitch + cx;
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
      for (int q = 0; q < 4; ++q) neumaier(s[k], cc[k], (double)buf[(q * 4 + k) * P + o]);
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) red[k][threadIdx.x] = s[k] + cc[k];
  __syncthreads();
  if (threadIdx.x < 4) {
    const int k = threadIdx.x;
    double ts = 0.0, tc = 0.0;
    for (int i = 0; i < 256; ++i) neumaier(ts, tc, red[k][i]);
    partial[4 * (int64_t)blockIdx.x + k] = ts + tc;
  }
}

hipError_t launch_audit(const void *buf, const Tile *tiles, int ntiles, int64_t plane,
                        int pitch, int fp32, double *partial, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  if (fp32)
    hipLaunchKernelGGL(audit_kernel<float>, dim3(ntiles), dim3(256), 0, s,
                       static_cast<const float *>(buf), tiles, plane, pitch, partial);
  else
    hipLaunchKernelGGL(audit_kernel<double>, dim3(ntiles), dim3(256), 0, s,
                       static_cast<const double *>(buf), tiles, plane, pitch, partial);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// State in / out
// ---------------------------------------------------------------------------
template <class T>
__global__ void set_kernel(RectArgs a, int raw) {
  const int64_t n = (int64_t)a.nx * a.ny;
  for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < n;
       c += (int64_t)gridDim.x * blockDim.x) {
    const int y = (int)(c / a.nx), x = (int)(c - (int64_t)y * a.nx);
    const int fx = a.x0 + x - a.fx0, sr = a.srow[a.y0 + y - a.fy0];
    if (sr < 0 || a.status[(int64_t)sr * a.fw + fx] == 0) continue;
    const int64_t o = (int64_t)sr * a.pitch + fx + a.xoff;
    double f[16];
    if (raw) {
#pragma unroll
      for (int i = 0; i < 16; ++i) f[i] = a.host_stage[i * n + c];
    } else {
      double W[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) W[k] = a.host_stage[k * n + c];
      equilibrium(W, a.eos, a.h, f);
    }
    T *b0 = static_cast<T *>(a.buf0), *b1 = static_cast<T *>(a.buf1);
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      b0[i * a.plane + o] = (T)f[i];
      b1[i * a.plane + o] = (T)f[i];
    }
  }
}

template <class T>
__global__ void get_kernel(RectArgs a, int pops) {
  const int64_t n = (int64_t)a.nx * a.ny;
  const double nan = __builtin_nan("");
  for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < n;
       c += (int64_t)gridDim.x * blockDim.x) {
    const int y = (int)(c / a.nx), x = (int)(c - (int64_t)y * a.nx);
    const int fx = a.x0 + x - a.fx0, sr = a.srow[a.y0 + y - a.fy0];
    const bool act = sr >= 0 && a.status[(int64_t)sr * a.fw + fx] == 1;
    const int64_t o = (int64_t)(sr < 0 ? 0 : sr) * a.pitch + fx + a.xoff;
    const T *b0 = static_cast<const T *>(a.buf0);
    if (pops) {
#pragma unroll
      for (int i = 0; i < 16; ++i) a.host_stage[i * n + c] = act ? (double)b0[i * a.plane + o] : nan;
    } else {
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        double w = nan;
        if (act)
          w = (((double)b0[(0 + k) * a.plane + o] + (double)b0[(4 + k) * a.plane + o]) +
               (double)b0[(8 + k) * a.plane + o]) +
              (double)b0[(12 + k) * a.plane + o];
        a.host_stage[k * n + c] = w;
      }
    }
  }
}

static dim3 grid_for(int64_t n) {
  int64_t g = (n + 255) / 256;
  if (g > 65535) g = 65535;
  if (g < 1) g = 1;
  return dim3((unsigned)g);
}

hipError_t launch_set_state(const RectArgs &a, int fp32, int raw, hipStream_t s) {
  const int64_t n = (int64_t)a.nx * a.ny;
  if (n == 0) return hipSuccess;
  if (fp32)
    hipLaunchKernelGGL(set_kernel<float>, grid_for(n), dim3(256), 0, s, a, raw);
  else
    hipLaunchKernelGGL(set_kernel<double>, grid_for(n), dim3(256), 0, s, a, raw);
  return hipGetLastError();
}

hipError_t launch_get(const RectArgs &a, int fp32, int pops, hipStream_t s) {
  const int64_t n = (int64_t)a.nx * a.ny;
  if (n == 0) return hipSuccess;
  if (fp32)
    hipLaunchKernelGGL(get_kernel<float>, grid_for(n), dim3(256), 0, s, a, pops);
  else
    hipLaunchKernelGGL(get_kernel<double>, grid_for(n), dim3(256), 0, s, a, pops);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Health scan: rho <= 0, p <= 0 or NaN on any active cell
// ---------------------------------------------------------------------------
template <class T>
__global__ void health_kernel(const T *__restrict__ buf, const Tile *tiles, int64_t P,
                              int pitch, EosT<double> eos, int *flag) {
  const Tile tl = tiles[blockIdx.x];
  const int n = tl.w * tl.h;
  int bad = 0;
  for (int c = threadIdx.x; c < n; c += blockDim.x) {
    const int cy = c / tl.w;
    const int cx = c - cy * tl.w;
    const int64_t o = (int64_t)tl.off0 + (int64_t)cy * pitch + cx;
    double W[4];
#pragma unroll
    for (int k = 0; k < 4; ++k)
      W[k] = (((double)buf[(0 + k) * P + o] + (double)buf[(4 + k) * P + o]) +
              (double)buf[(8 + k) * P + o]) +
             (double)buf[(12 + k) * P + o];
    const double u = W[1] / W[0], v = W[2] / W[0];
    const double p = pressure<double>(eos, W[0], W[3] - 0.5 * (W[1] * u + W[2] * v));
    if (!(W[0] > 0.0) || !(p > 0.0)) bad = 1;
  }
  if (bad) atomicOr(flag, 1);
}

hipError_t launch_health(const void *buf, const Tile *tiles, int ntiles, int64_t plane,
                         int pitch, int fp32, const EosT<double> &eos, int *flag, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  if (fp32)
    hipLaunchKernelGGL(health_kernel<float>, dim3(ntiles), dim3(256), 0, s,
                       static_cast<const float *>(buf), tiles, plane, pitch, eos, flag);
  else
    hipLaunchKernelGGL(health_kernel<double>, dim3(ntiles), dim3(256), 0, s,
                       static_cast<const double *>(buf), tiles, plane, pitch, eos, flag);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Density-gradient tags on active cells of one level
// ---------------------------------------------------------------------------
template <class T>
__device__ __forceinline__ double cell_rho(const T *b, int64_t P, int64_t o) {
  return (((double)b[0 * P + o] + (double)b[4 * P + o]) + (double)b[8 * P + o]) +
         (double)b[12 * P + o];
}

// Density of every stored frame cell (0 where it is not an active cell), in
// FP64 from the stored populations, indexed like the status.
template <class T>
__global__ void rho_kernel(const T *__restrict__ buf, const uint8_t *__restrict__ status, int64_t P, int pitch,
                           int xoff, int fw, int nrows, double *__restrict__ rho) {
  // x: frame column, y: stored rows (strided when there are more than the grid)
  const int fx = blockIdx.x * blockDim.x + threadIdx.x;
  if (fx >= fw) return;
  for (int sr = blockIdx.y; sr < nrows; sr += gridDim.y) {
    const int64_t c = (int64_t)sr * fw + fx;
    rho[c] = status[c] == 1 ? cell_rho<T>(buf, P, (int64_t)sr * pitch + fx + xoff) : 0.0;
  }
}

// Density-gradient tags from the density plane (rho_kernel): each density is
// summed once, and a cell's four neighbours read theirs from the plane.
__global__ void tag_kernel(const double *__restrict__ rho, const uint8_t *__restrict__ status,
                           const int32_t *__restrict__ srow, const int32_t *__restrict__ yrow, int fx0, int fy0,
                           int fw, int fh, int nrows, int Nx, int Ny, int perx, int pery, double thr,
                           uint8_t *__restrict__ tags) {
  // one thread per stored frame cell (x: frame column, y: stored rows); tags
  // are indexed like the status (only active cells of the level, which all
  // lie in its frame, can be tagged)
  const int fx = blockIdx.x * blockDim.x + threadIdx.x;
  if (fx >= fw) return;
  for (int sr = blockIdx.y; sr < nrows; sr += gridDim.y) {
    const int64_t c = (int64_t)sr * fw + fx;
    const int x = fx + fx0, y = yrow[sr] + fy0;
    // every load issued up front: a neighbour's status and density are read
    // at once (the density of an inactive neighbour is read and not used)
    const uint8_t sc = status[c];
    const double rc = rho[c];
    const int dx[4] = {1, -1, 0, 0}, dy[4] = {0, 0, 1, -1};
    int64_t ni[4];
    bool valid[4];
#pragma unroll
    for (int d = 0; d < 4; ++d) {
      int xx = x + dx[d], yy = y + dy[d];
      bool ok = true;
      if (xx < 0 || xx >= Nx) {
        if (perx) xx = (xx + Nx) % Nx; else ok = false;
      }
      if (yy < 0 || yy >= Ny) {
        if (pery) yy = (yy + Ny) % Ny; else ok = false;
      }
      const int gx = xx - fx0, gy = yy - fy0;
      // the same stored row for a neighbour along x
      const int gs = !ok ? -1 : dy[d] == 0 ? sr : (gy >= 0 && gy < fh) ? srow[gy] : -1;
      valid[d] = gs >= 0 && gx >= 0 && gx < fw;
      ni[d] = valid[d] ? (int64_t)gs * fw + gx : c;
    }
    uint8_t sn[4];
    double rv[4];
#pragma unroll
    for (int d = 0; d < 4; ++d) {
      sn[d] = status[ni[d]];
      rv[d] = rho[ni[d]];
    }
    uint8_t tag = 0;
    if (sc == 1) {
      double rn[4];
#pragma unroll
      for (int d = 0; d < 4; ++d) rn[d] = (valid[d] && sn[d] == 1) ? rv[d] : rc;
      const double gx = fabs(rn[0] - rn[1]) / (2.0 * rc);
      const double gy = fabs(rn[2] - rn[3]) / (2.0 * rc);
      const double g = gx > gy ? gx : gy;
      tag = (uint8_t)(g > thr);
    }
    tags[c] = tag;
  }
}

hipError_t launch_tag(const void *buf, const uint8_t *status, const int32_t *srow, const int32_t *yrow,
                      int64_t plane, int pitch, int xoff, int fx0, int fy0, int fw, int fh, int nrows,
                      int Nx, int Ny, int perx, int pery, int fp32, double thr, double *rho, uint8_t *tags,
                      hipStream_t s) {
  const int64_t n = (int64_t)fw * nrows;
  if (n <= 0) return hipSuccess;
  const dim3 grid((unsigned)((fw + 255) / 256), (unsigned)std::min(nrows, 65535));
  if (fp32)
    hipLaunchKernelGGL(rho_kernel<float>, grid, dim3(256), 0, s, static_cast<const float *>(buf), status, plane,
                       pitch, xoff, fw, nrows, rho);
  else
    hipLaunchKernelGGL(rho_kernel<double>, grid, dim3(256), 0, s, static_cast<const double *>(buf), status, plane,
                       pitch, xoff, fw, nrows, rho);
  hipLaunchKernelGGL(tag_kernel, grid, dim3(256), 0, s, rho, status, srow, yrow, fx0, fy0, fw, fh, nrows, Nx, Ny,
                     perx, pery, thr, tags);
  return hipGetLastError();
}

// Refinement sensor of eq. amr-sigma (Sec. 3.4). First the domain-wide
// max_{x,alpha} |Q_{alpha,k}| over the active cells of every level (one
// launch per level over its step tiles, into qmax as bits), then per active
// cell s_k = (0.5 ((Qx_k(x+1) - Qx_k(x-1)) + (Qy_k(y+1) - Qy_k(y-1)))) / qmax_k
// (0 where qmax_k is 0), a neighbour that is not an active cell replaced by
// the cell itself, and the tag max_k |s_k| > thr. The arithmetic follows the
// order of the FP64 contract above.
template <class T>
__global__ __launch_bounds__(256) void flux_max_kernel(const T *__restrict__ buf, const Tile *tiles, int64_t P,
                                                       int pitch, EosT<double> eos, unsigned long long *qmax) {
  const Tile tl = tiles[blockIdx.x];
  double m[4] = {0.0, 0.0, 0.0, 0.0};
  const int n = tl.w * tl.h;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const int cy = i / tl.w, cx = i - cy * tl.w;
    double w[4];
    stored_W<T>(buf, P, (int64_t)tl.off0 + (int64_t)cy * pitch + cx, w);
    flux_absmax(eos, w, m);
  }
  block_qmax(m, qmax);
}

hipError_t launch_flux_max(const void *buf, const Tile *tiles, int ntiles, int64_t plane, int pitch, int fp32,
                           const EosT<double> &eos, unsigned long long *qmax, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  if (fp32)
    hipLaunchKernelGGL(flux_max_kernel<float>, dim3(ntiles), dim3(256), 0, s, static_cast<const float *>(buf),
                       tiles, plane, pitch, eos, qmax);
  else
    hipLaunchKernelGGL(flux_max_kernel<double>, dim3(ntiles), dim3(256), 0, s, static_cast<const double *>(buf),
                       tiles, plane, pitch, eos, qmax);
  return hipGetLastError();
}

template <class T>
__global__ void tag_flux_kernel(const T *__restrict__ buf, const uint8_t *status, const int32_t *srow,
                                const int32_t *yrow, int64_t P, int pitch, int xoff, int fx0, int fy0, int fw,
                                int fh, int nrows, int Nx, int Ny, int perx, int pery, EosT<double> eos,
                                const unsigned long long *qmax_bits, double thr, uint8_t *tags) {
  const int64_t n = (int64_t)fw * nrows;
  double qm[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) qm[k] = __longlong_as_double((long long)qmax_bits[k]);
  for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < n;
       c += (int64_t)gridDim.x * blockDim.x) {
    const int sr = (int)(c / fw), fx = (int)(c - (int64_t)sr * fw);
    const int x = fx + fx0, y = yrow[sr] + fy0;
    uint8_t tag = 0;
    if (status[c] == 1) {
      const int64_t o = (int64_t)sr * pitch + fx + xoff;
      const int dx[4] = {1, -1, 0, 0}, dy[4] = {0, 0, 1, -1};
      double Qx[4][4], Qy[4][4];
#pragma unroll
      for (int d = 0; d < 4; ++d) {
        int xx = x + dx[d], yy = y + dy[d];
        bool ok = true;
        if (xx < 0 || xx >= Nx) {
          if (perx) xx = (xx + Nx) % Nx; else ok = false;
        }
        if (yy < 0 || yy >= Ny) {
          if (pery) yy = (yy + Ny) % Ny; else ok = false;
        }
        int64_t on = o;
        if (ok) {
          const int gx = xx - fx0, gy = yy - fy0;
          const int gs = (gy >= 0 && gy < fh) ? srow[gy] : -1;
          if (gx >= 0 && gx < fw && gs >= 0 && status[(int64_t)gs * fw + gx] == 1)
            on = (int64_t)gs * pitch + gx + xoff;
        }
        double w[4];
        stored_W<T>(buf, P, on, w);
        euler_flux(eos, w, Qx[d], Qy[d]);
      }
      double smax = 0.0;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const double dq = (Qx[0][k] - Qx[1][k]) + (Qy[2][k] - Qy[3][k]);
        const double sk = qm[k] > 0.0 ? (0.5 * dq) / qm[k] : 0.0;
        smax = fabs(sk) > smax ? fabs(sk) : smax;
      }
      tag = (uint8_t)(smax > thr);
    }
    tags[c] = tag;
  }
}

hipError_t launch_tag_flux(const void *buf, const uint8_t *status, const int32_t *srow, const int32_t *yrow,
                           int64_t plane, int pitch, int xoff, int fx0, int fy0, int fw, int fh, int nrows, int Nx,
                           int Ny, int perx, int pery, int fp32, const EosT<double> &eos,
                           const unsigned long long *qmax, double thr, uint8_t *tags, hipStream_t s) {
  const int64_t n = (int64_t)fw * nrows;
  if (n <= 0) return hipSuccess;
  if (fp32)
    hipLaunchKernelGGL(tag_flux_kernel<float>, grid_for(n), dim3(256), 0, s, static_cast<const float *>(buf),
                       status, srow, yrow, plane, pitch, xoff, fx0, fy0, fw, fh, nrows, Nx, Ny, perx, pery, eos,
                       qmax, thr, tags);
  else
    hipLaunchKernelGGL(tag_flux_kernel<double>, grid_for(n), dim3(256), 0, s, static_cast<const double *>(buf),
                       status, srow, yrow, plane, pitch, xoff, fx0, fy0, fw, fh, nrows, Nx, Ny, perx, pery, eos,
                       qmax, thr, tags);
  return hipGetLastError();
}

// Refined features keep their levels: every tagged cell of a level-(l+1)
// frame tags its parent in the level-l frame (one thread per stored fine frame
// cell; several children write the same 1, which is benign).
__global__ void tag_parents_kernel(const uint8_t *__restrict__ ftags, const int32_t *__restrict__ fyrow,
                                   int ffx0, int ffy0, int ffw, int fnrows, uint8_t *__restrict__ ptags,
                                   const int32_t *__restrict__ psrow, int pfx0, int pfy0, int pfw, int pfh,
                                   int r) {
  const int64_t n = (int64_t)ffw * fnrows;
  for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < n;
       c += (int64_t)gridDim.x * blockDim.x) {
    if (!ftags[c]) continue;
    const int sr = (int)(c / ffw), fx = (int)(c - (int64_t)sr * ffw);
    const int x = ffx0 + fx, y = ffy0 + fyrow[sr];  // a tagged cell is active, hence in the domain
    const int px = x / r - pfx0, py = y / r - pfy0;
    if (px < 0 || px >= pfw || py < 0 || py >= pfh) continue;
    const int ps = psrow[py];
    if (ps >= 0) ptags[(int64_t)ps * pfw + px] = 1;
  }
}

hipError_t launch_tag_parents(const uint8_t *ftags, const int32_t *fyrow, int ffx0, int ffy0, int ffw,
                              int fnrows, uint8_t *ptags, const int32_t *psrow, int pfx0, int pfy0, int pfw,
                              int pfh, int r, hipStream_t s) {
  const int64_t n = (int64_t)ffw * fnrows;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(tag_parents_kernel, grid_for(n), dim3(256), 0, s, ftags, fyrow, ffx0, ffy0, ffw, fnrows,
                     ptags, psrow, pfx0, pfy0, pfw, pfh, r);
  return hipGetLastError();
}

// Tiles of the clustering grid (side T level cells, ntx tiles per tile row)
// that hold a cell within `buf` cells of a tag (square dilation, periodic axes
// wrapped, other axes clipped), in two passes: the rows' tag masks, then per
// tile a range test of each of its window rows.
//
// Row masks of the tags: bit j of word w of stored frame row sr is the tag of
// level column 64 w + j (0 outside the frame). One thread per level column,
// 64 columns per wavefront (one word each).
__global__ void row_mask_kernel(const uint8_t *__restrict__ tags, int fx0, int fw, int nrows, int Nx, int nw,
                                unsigned long long *__restrict__ masks) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t per_row = (int64_t)nw * 64;
  bool bit = false;
  int64_t word = -1;
  if (t < (int64_t)nrows * per_row) {
    const int sr = (int)(t / per_row), x = (int)(t - (int64_t)sr * per_row);
    word = (int64_t)sr * nw + (x >> 6);
    const int fx = x - fx0;
    bit = x < Nx && fx >= 0 && fx < fw && tags[(int64_t)sr * fw + fx] != 0;
  }
  const unsigned long long m = __ballot(bit);
  if ((threadIdx.x & 63) == 0 && word >= 0) masks[word] = m;
}

// Any set bit of row mask mr in columns [xa, xb), 0 <= xa < xb.
__device__ __forceinline__ bool any_bits(const unsigned long long *mr, int xa, int xb) {
  unsigned long long acc = 0;
  for (int w = xa >> 6; w <= (xb - 1) >> 6; ++w) {
    const int lo = w == (xa >> 6) ? (xa & 63) : 0, hi = w == ((xb - 1) >> 6) ? ((xb - 1) & 63) : 63;
    const unsigned long long sel = (hi == 63 ? ~0ull : ((1ull << (hi + 1)) - 1ull)) & ~((1ull << lo) - 1ull);
    acc |= mr[w] & sel;
  }
  return acc != 0;
}

// Tiles of side T (level cells) that hold a cell within `buf` of a tag: one
// thread per tile of the listed tile rows tests its window
// [x0 - buf, x1 + buf) x [y0 - buf, y1 + buf) row by row on the row masks
// (periodic axes wrapped, other axes clipped); the hits of a wavefront are
// appended with one atomic, the list in no particular order (at most cap
// entries stored).
__global__ void tile_hits_kernel(const unsigned long long *__restrict__ masks, int nw, const int32_t *__restrict__ srow,
                                 int fy0, int fh, int Nx, int Ny, int perx, int pery, int T, int buf, int ntx,
                                 const int32_t *__restrict__ trows, int ntrows, int32_t *list, int cap, int *count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool hit = false;
  int32_t t = 0;
  if (i < (int64_t)ntrows * ntx) {
    const int ty = trows[i / ntx], tx = (int)(i % ntx);
    t = ty * ntx + tx;
    const int x0 = tx * T, x1 = min(Nx, x0 + T);
    const int xa = x0 - buf, xb = x1 + buf;
    const int ya = ty * T - buf, yb = min(Ny, ty * T + T) + buf;
    for (int y = ya; y < yb; ++y) {
      int wy = y;
      if (wy < 0 || wy >= Ny) {
        if (!pery) continue;
        wy = wy < 0 ? wy + Ny : wy - Ny;
      }
      const int fr = wy - fy0;
      if (fr < 0 || fr >= fh) continue;
      const int sr = srow[fr];
      if (sr < 0) continue;
      const unsigned long long *mr = masks + (int64_t)sr * nw;
      bool h;
      if (!perx) {
        h = any_bits(mr, max(0, xa), min(Nx, xb));
      } else if (xb - xa >= Nx) {
        h = any_bits(mr, 0, Nx);
      } else if (xa < 0) {
        h = any_bits(mr, xa + Nx, Nx) || any_bits(mr, 0, xb);
      } else if (xb > Nx) {
        h = any_bits(mr, xa, Nx) || any_bits(mr, 0, xb - Nx);
      } else {
        h = any_bits(mr, xa, xb);
      }
      hit = hit || h;
    }
  }
  const unsigned long long m = __ballot(hit);
  if (!m) return;
  const int lane = (int)(threadIdx.x & 63);
  const int leader = __ffsll((long long)m) - 1;
  int base = 0;
  if (lane == leader) base = atomicAdd(count, __popcll(m));
  base = __shfl(base, leader);
  if (hit) {
    const int at = base + __popcll(m & ((1ull << lane) - 1ull));
    if (at < cap) list[at] = t;
  }
}

hipError_t launch_tile_hits(const uint8_t *tags, const int32_t *srow, int fx0, int fy0, int fw, int fh, int nrows,
                            int Nx, int Ny, int perx, int pery, int T, int buf, int ntx, const int32_t *trows,
                            int ntrows, unsigned long long *masks, int32_t *list, int cap, int *count, hipStream_t s) {
  const int nw = (Nx + 63) / 64;
  const int64_t nm = (int64_t)nrows * nw * 64;
  if (nm > 0)
    hipLaunchKernelGGL(row_mask_kernel, dim3((unsigned)((nm + 255) / 256)), dim3(256), 0, s, tags, fx0, fw, nrows,
                       Nx, nw, masks);
  const int64_t n = (int64_t)ntrows * ntx;
  if (n <= 0) return hipGetLastError();
  hipLaunchKernelGGL(tile_hits_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, masks, nw, srow, fy0, fh,
                     Nx, Ny, perx, pery, T, buf, ntx, trows, ntrows, list, cap, count);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Regrid: merge (eq. amr-merge) and minmod split (eqs. amr-slope, amr-split)
// One thread per (operation, population plane).
// ---------------------------------------------------------------------------
template <class T>
__global__ void merge_kernel(RegridArgs a) {
  const int64_t n = (int64_t)a.nops * 16;
  const T *F = static_cast<const T *>(a.fine_cur ? a.fine1 : a.fine0);
  T *C0 = static_cast<T *>(a.coarse0), *C1 = static_cast<T *>(a.coarse1);
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n;
       t += (int64_t)gridDim.x * blockDim.x) {
    const RegridOp op = a.ops[t >> 4];
    const int i = (int)(t & 15);
    double s = 0.0;
    for (int bb = 0; bb < a.r; ++bb)
      for (int aa = 0; aa < a.r; ++aa)
        s += (double)F[i * a.fplane + op.src + (int64_t)bb * a.fpitch + aa];
    const double m = s / (double)(a.r * a.r);
    C0[i * a.cplane + op.dst] = (T)m;
    C1[i * a.cplane + op.dst] = (T)m;
  }
}

template <class T>
__global__ void split_kernel(RegridArgs a) {
  const int64_t n = (int64_t)a.nops * 16;
  const T *C = static_cast<const T *>(a.coarse_cur ? a.coarse1 : a.coarse0);
  T *F0 = static_cast<T *>(a.fine0), *F1 = static_cast<T *>(a.fine1);
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n;
       t += (int64_t)gridDim.x * blockDim.x) {
    const RegridOp op = a.ops[t >> 4];
    const int i = (int)(t & 15);
    const int64_t pl = i * a.cplane;
    const double fi = (double)C[pl + op.src];
    double sx = 0.0, sy = 0.0;
    if (op.nb[1] >= 0 && op.nb[0] >= 0)
      sx = minmod(fi - (double)C[pl + op.nb[1]], (double)C[pl + op.nb[0]] - fi);
    if (op.nb[3] >= 0 && op.nb[2] >= 0)
      sy = minmod(fi - (double)C[pl + op.nb[3]], (double)C[pl + op.nb[2]] - fi);
    for (int bb = 0; bb < a.r; ++bb)
      for (int aa = 0; aa < a.r; ++aa) {
        const double xa = (double)(2 * aa - a.r + 1) / (double)(2 * a.r);
        const double xb = (double)(2 * bb - a.r + 1) / (double)(2 * a.r);
        double v = fi + sx * xa;
        v = v + sy * xb;
        const int64_t o = i * a.fplane + op.dst + (int64_t)bb * a.fpitch + aa;
        F0[o] = (T)v;
        F1[o] = (T)v;
      }
  }
}

hipError_t launch_merge(const RegridArgs &a, int fp32, hipStream_t s) {
  if (a.nops <= 0) return hipSuccess;
  const int64_t n = (int64_t)a.nops * 16;
  if (fp32)
    hipLaunchKernelGGL(merge_kernel<float>, grid_for(n), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL(merge_kernel<double>, grid_for(n), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_split(const RegridArgs &a, int fp32, hipStream_t s) {
  if (a.nops <= 0) return hipSuccess;
  const int64_t n = (int64_t)a.nops * 16;
  if (fp32)
    hipLaunchKernelGGL(split_kernel<float>, grid_for(n), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL(split_kernel<double>, grid_for(n), dim3(256), 0, s, a);
  return hipGetLastError();
}

// Copy whole cells (16 planes) between two frames: pairs[2i] source offset,
// pairs[2i+1] destination offset.
template <class T>
__global__ void copy_cells_kernel(const T *__restrict__ src, T *__restrict__ dst,
                                  const int32_t *pairs, int npairs, int64_t sp, int64_t dp) {
  const int64_t n = (int64_t)npairs * 16;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t p = t >> 4;
    const int i = (int)(t & 15);
    dst[i * dp + pairs[2 * p + 1]] = src[i * sp + pairs[2 * p]];
  }
}

hipError_t launch_copy_frame(const void *src, void *dst, const int32_t *pairs, int npairs,
                             int64_t splane, int64_t dplane, int fp32, hipStream_t s) {
  if (npairs <= 0) return hipSuccess;
  const int64_t n = (int64_t)npairs * 16;
  if (fp32)
    hipLaunchKernelGGL(copy_cells_kernel<float>, grid_for(n), dim3(256), 0, s,
                       static_cast<const float *>(src), static_cast<float *>(dst), pairs, npairs,
                       splane, dplane);
  else
    hipLaunchKernelGGL(copy_cells_kernel<double>, grid_for(n), dim3(256), 0, s,
                       static_cast<const double *>(src), static_cast<double *>(dst), pairs,
                       npairs, splane, dplane);
  return hipGetLastError();
}

// New interfaces after a regrid: population q of each listed ring cell gets
// its current value in the level's other buffer too (items[2i] element
// offset, items[2i+1] q), so the first hand-off across that face is flat.
template <class T>
__global__ void restart_faces_kernel(const T *__restrict__ cur, T *__restrict__ other,
                                     const int32_t *items, int n, int64_t P) {
  const int64_t total = (int64_t)n * 4;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = t >> 2;
    const int k = (int)(t & 3);
    const int64_t e = (int64_t)(items[2 * i + 1] * 4 + k) * P + items[2 * i];
    other[e] = cur[e];
  }
}

hipError_t launch_restart_faces(const void *cur, void *other, const int32_t *items, int n,
                                int64_t plane, int fp32, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t total = (int64_t)n * 4;
  if (fp32)
    hipLaunchKernelGGL(restart_faces_kernel<float>, grid_for(total), dim3(256), 0, s,
                       static_cast<const float *>(cur), static_cast<float *>(other), items, n, plane);
  else
    hipLaunchKernelGGL(restart_faces_kernel<double>, grid_for(total), dim3(256), 0, s,
                       static_cast<const double *>(cur), static_cast<double *>(other), items, n, plane);
  return hipGetLastError();
}

}  // namespace vlbm
