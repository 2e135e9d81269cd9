// Device code of the three-dimensional (D3Q6) path of libvlbm, gfx950.
// Storage S (double, or float for the FP32 forms) and arithmetic type C of the
// cell update (double, or float for plain FP32); hand-off, reflux, ledger,
// audit and regrid arithmetic is FP64 in every form, rounded to S on store.
//
// `step3_kernel`: one workgroup per tile of active cells. It first executes the
// tile's ghost and interface tasks (slots only its own cells read, reflux
// captures), then, after one workgroup barrier, advances every cell: pull the
// six inbound populations (exact shift, Sec. 2.2), relax them towards the
// vectorial equilibrium (eqs. num-equilibrium with D = 3, num-relaxation) and
// store the 30 post-collision values. Structure-of-arrays planes make every
// load and store of a wavefront a contiguous run along x.
//
// Arithmetic contract (the oracle's order; built with -ffp-contract=off):
//   W_k = ((((f_{0k} + f_{1k}) + f_{2k}) + f_{3k}) + f_{4k}) + f_{5k}
//   u = m_x / rho, v = m_y / rho, w = m_z / rho
//   p = (gamma - 1) (E - 0.5 ((m_x u + m_y v) + m_z w))
//   Q_x = (m_x, m_x u + p, m_y u, m_z u, (E + p) u), Q_y, Q_z alike
//   f^eq_{+-alpha,k} = W_k / 6 +- h Q_{alpha,k},  h = 1 / (2c)
//   f*_{qk} = f_{qk} + 2 beta (f^eq_{qk} - f_{qk})
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>

#include "vlbm3_internal.hpp"

namespace vlbm3 {

template <class S>
using g1 = __attribute__((address_space(1))) S *;

template <class C>
__device__ __forceinline__ void relax3(C g[30], C gm1, C h, C tb) {
  C W[5];
#pragma unroll
  for (int k = 0; k < 5; ++k)
    W[k] = ((((g[k] + g[5 + k]) + g[10 + k]) + g[15 + k]) + g[20 + k]) + g[25 + k];
  const C rho = W[0], mx = W[1], my = W[2], mz = W[3], E = W[4];
  const C u = mx / rho;
  const C v = my / rho;
  const C w = mz / rho;
  const C p = gm1 * (E - C(0.5) * ((mx * u + my * v) + mz * w));
  const C Q[3][5] = {{mx, mx * u + p, my * u, mz * u, (E + p) * u},
                     {my, mx * v, my * v + p, mz * v, (E + p) * v},
                     {mz, mx * w, my * w, mz * w + p, (E + p) * w}};
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    const C share = W[k] / C(6);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const C hq = h * Q[a][k];
      C &fp = g[(2 * a) * 5 + k];
      C &fm = g[(2 * a + 1) * 5 + k];
      fp = fp + tb * ((share + hq) - fp);
      fm = fm + tb * ((share - hq) - fm);
    }
  }
}

__device__ __forceinline__ double minmod3(double a, double b) {
  if (a > 0.0 && b > 0.0) return a < b ? a : b;
  if (a < 0.0 && b < 0.0) return a > b ? a : b;
  return 0.0;
}

template <class T>
__device__ __forceinline__ void run_task3(const Desc3 &A, int first, double ak, const Task3 &t) {
  T *S = static_cast<T *>(A.src);
  const int64_t P = A.plane;
  const int q = t.q;
  switch (t.kind & 0xFF) {
    case K3_COPY:
#pragma unroll
      for (int k = 0; k < 5; ++k) S[(q * 5 + k) * P + t.dst] = S[(q * 5 + k) * P + t.src];
      break;
    case K3_OUTFLOW:
    case K3_REFLECT: {
      const int qo = q ^ 1;
      const int kn = 1 + (q >> 1);  // momentum component along the side's normal
      const bool refl = (t.kind & 0xFF) == K3_REFLECT;
      const bool book = (t.kind & K3_LEDGER) != 0;
      double *L = A.ledger + 5 * (int64_t)t.slot;
#pragma unroll
      for (int k = 0; k < 5; ++k) {
        double vin;
        if (refl) {
          const double w = (double)S[(qo * 5 + k) * P + t.src];
          vin = (k == kn) ? -w : w;
        } else {
          vin = (double)S[(q * 5 + k) * P + t.src];
        }
        S[(q * 5 + k) * P + t.dst] = (T)vin;
        if (book) {
          const double out = (double)S[(qo * 5 + k) * P + t.src];
          const double l = L[k] + A.w3 * vin;
          L[k] = l + (-1.0) * (A.w3 * out);
        }
      }
      break;
    }
    case K3_RECON: {
      const T *C = static_cast<const T *>(A.pcur);
      const T *Pv = static_cast<const T *>(A.pprev);
      const int64_t P2 = A.pplane;
      const double b1 = (double)(2 * t.j1 - A.r + 1) / (double)(2 * A.r);
      const double b2 = (double)(2 * t.j2 - A.r + 1) / (double)(2 * A.r);
#pragma unroll
      for (int k = 0; k < 5; ++k) {
        const int64_t pl = (q * 5 + k) * P2;
        const double out = (double)C[pl + t.src];
        const double prev = (double)Pv[pl + t.src];
        double v = out + (out - prev) * ak;
        const double s1 =
            (t.n[0] >= 0) ? minmod3(out - (double)C[pl + t.n[0]], (double)C[pl + t.n[1]] - out) : 0.0;
        v = v + s1 * b1;
        const double s2 =
            (t.n[2] >= 0) ? minmod3(out - (double)C[pl + t.n[2]], (double)C[pl + t.n[3]] - out) : 0.0;
        v = v + s2 * b2;
        S[(q * 5 + k) * P + t.dst] = (T)v;
      }
      break;
    }
    case K3_REFLUX:
#pragma unroll
      for (int k = 0; k < 5; ++k) S[(q * 5 + k) * P + t.dst] = (T)(A.acc_in[5 * (int64_t)t.slot + k] / A.rrr);
      break;
    case K3_CAPTURE: {
      double *acc = A.acc_out + 5 * (int64_t)t.slot;
      const int r = A.r;
#pragma unroll
      for (int k = 0; k < 5; ++k) {
        double s = first ? 0.0 : acc[k];
        const int64_t base = (q * 5 + k) * P + t.src;
        for (int a = 0; a < r; ++a)
          for (int b = 0; b < r; ++b) s = s + (double)S[base + (int64_t)a * t.n[0] + (int64_t)b * t.n[1]];
        acc[k] = s;
      }
      break;
    }
    default:
      break;
  }
}

template <class S, class C, bool NT>
__global__ __launch_bounds__(256) void step3_kernel(Launch3 L) {
  const Desc3 &A = *L.d;
  const int tid = blockIdx.x;
  // everything the cell loop needs is read before the first store
  const int ntiles = A.ntiles;
  if (tid >= ntiles) return;
  const Tile3 tl = A.tiles[tid];
  const auto s = (g1<const S>)A.src;
  const auto d = (g1<S>)A.dst;
  const int64_t P = A.plane, slab = A.slab;
  const int pitch = A.pitch;
  const C gm1 = (C)A.gm1, h = (C)A.h, tb = (C)A.tb;
  if (tl.ntask) {
    for (int i = threadIdx.x; i < tl.ntask; i += blockDim.x)
      run_task3<S>(A, L.first, L.ak, A.tasks[tl.task0 + i]);
    __syncthreads();
  }
  const int n = tl.w * tl.h;
  for (int c = threadIdx.x; c < n; c += blockDim.x) {
    const int cy = c / tl.w, cx = c - cy * tl.w;
    const int64_t o = (int64_t)tl.off0 + (int64_t)cy * pitch + cx;
    C g[30];
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      g[k] = (C)s[(0 * 5 + k) * P + o - 1];            // +x arrives from x - 1
      g[5 + k] = (C)s[(1 * 5 + k) * P + o + 1];        // -x from x + 1
      g[10 + k] = (C)s[(2 * 5 + k) * P + o - pitch];   // +y from y - 1
      g[15 + k] = (C)s[(3 * 5 + k) * P + o + pitch];   // -y from y + 1
      g[20 + k] = (C)s[(4 * 5 + k) * P + o - slab];    // +z from z - 1
      g[25 + k] = (C)s[(5 * 5 + k) * P + o + slab];    // -z from z + 1
    }
    relax3<C>(g, gm1, h, tb);
#pragma unroll
    for (int i = 0; i < 30; ++i) {
      const S v = (S)g[i];
      if (NT)
        __builtin_nontemporal_store(v, &d[i * P + o]);
      else
        d[i * P + o] = v;
    }
  }
}

hipError_t launch_step3(const Launch3 &a, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
  if (a.nblocks <= 0) return hipSuccess;
  const dim3 grid(a.nblocks), block(256);
  const bool nt = (a.flags & S3_NT_STORES) != 0;
#define VLBM3_STEP(S_, C_)                                                                        \
  do {                                                                                            \
    if (nt)                                                                                       \
      hipExtLaunchKernelGGL((step3_kernel<S_, C_, true>), grid, block, 0, s, ev0, ev1, 0, a);      \
    else                                                                                          \
      hipExtLaunchKernelGGL((step3_kernel<S_, C_, false>), grid, block, 0, s, ev0, ev1, 0, a);     \
  } while (0)
  if (!(a.flags & S3_FP32))
    VLBM3_STEP(double, double);
  else if (a.flags & S3_F64_MATH)
    VLBM3_STEP(float, double);
  else
    VLBM3_STEP(float, float);
#undef VLBM3_STEP
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Refinement tags (Sec. 3.4, density-gradient variant): an active cell is
// tagged when max over the axes of |rho(+1) - rho(-1)| / (2 rho) exceeds the
// threshold; a neighbour that is not an active cell of the level (across a
// non-periodic side, outside the frame, a hole, uncovered) stands in as the
// cell itself. rho = sum_q f_{q,rho} in the fixed order.
// ---------------------------------------------------------------------------
template <class T>
__device__ __forceinline__ double rho3(const T *b, int64_t P, int64_t o) {
  return (((((double)b[0 * P + o] + (double)b[5 * P + o]) + (double)b[10 * P + o]) + (double)b[15 * P + o]) +
          (double)b[20 * P + o]) +
         (double)b[25 * P + o];
}

template <class T>
__global__ __launch_bounds__(256) void tag3_kernel(Tag3Args a) {
  const int64_t n = (int64_t)a.fn[0] * a.fn[1] * a.fn[2];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int fx = (int)(i % a.fn[0]), fy = (int)((i / a.fn[0]) % a.fn[1]), fz = (int)(i / ((int64_t)a.fn[0] * a.fn[1]));
  if (a.status[i] != 1) {
    a.tags[i] = 0;
    return;
  }
  const T *b = static_cast<const T *>(a.buf);
  const int64_t o = (int64_t)fz * a.slab + (int64_t)fy * a.pitch + fx + a.xoff;
  const double rc = rho3(b, a.plane, o);
  const int fc[3] = {fx, fy, fz};
  double g = 0.0;
  for (int ax = 0; ax < 3; ++ax) {
    double side[2];
    for (int sd = 0; sd < 2; ++sd) {
      int q[3] = {a.f0[0] + fx, a.f0[1] + fy, a.f0[2] + fz};
      q[ax] += sd == 0 ? 1 : -1;
      bool ok = true;
      if (q[ax] < 0 || q[ax] >= a.N[ax]) {
        if ((a.periodic >> ax) & 1)
          q[ax] = q[ax] < 0 ? q[ax] + a.N[ax] : q[ax] - a.N[ax];
        else
          ok = false;
      }
      int gq[3] = {fc[0], fc[1], fc[2]};
      if (ok) {
        for (int k = 0; k < 3; ++k) {
          gq[k] = q[k] - a.f0[k];
          ok = ok && gq[k] >= 0 && gq[k] < a.fn[k];
        }
      }
      if (ok) ok = a.status[((int64_t)gq[2] * a.fn[1] + gq[1]) * a.fn[0] + gq[0]] == 1;
      side[sd] = ok ? rho3(b, a.plane, (int64_t)gq[2] * a.slab + (int64_t)gq[1] * a.pitch + gq[0] + a.xoff) : rc;
    }
    const double ga = fabs(side[0] - side[1]) / (2.0 * rc);
    if (ga > g) g = ga;
  }
  a.tags[i] = (uint8_t)(g > a.thr);
}

hipError_t launch_tag3(const Tag3Args &a, int fp32, hipStream_t s) {
  const int64_t n = (int64_t)a.fn[0] * a.fn[1] * a.fn[2];
  if (n <= 0) return hipSuccess;
  const dim3 grid((unsigned)((n + 255) / 256));
  if (fp32)
    hipLaunchKernelGGL(tag3_kernel<float>, grid, dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL(tag3_kernel<double>, grid, dim3(256), 0, s, a);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Conservation audit: per-tile compensated sums of sum_q f_{q,k}
// ---------------------------------------------------------------------------
__device__ __forceinline__ void neumaier3(double &s, double &c, double v) {
  const double t = s + v;
  if (fabs(s) >= fabs(v))
    c += (s - t) + v;
  else
    c += (v - t) + s;
  s = t;
}

template <class T>
__global__ __launch_bounds__(256) void audit3_kernel(const T *__restrict__ buf, const Tile3 *tiles,
                                                     int64_t P, int pitch, double *partial) {
  __shared__ double red[5][256];
  const Tile3 tl = tiles[blockIdx.x];
  double sm[5] = {0, 0, 0, 0, 0}, cc[5] = {0, 0, 0, 0, 0};
  const int n = tl.w * tl.h;
  for (int c = threadIdx.x; c < n; c += blockDim.x) {
    const int cy = c / tl.w, cx = c - cy * tl.w;
    const int64_t o = (int64_t)tl.off0 + (int64_t)cy * pitch + cx;
#pragma unroll
    for (int k = 0; k < 5; ++k)
#pragma unroll
      for (int q = 0; q < 6; ++q) neumaier3(sm[k], cc[k], (double)buf[(q * 5 + k) * P + o]);
  }
#pragma unroll
  for (int k = 0; k < 5; ++k) red[k][threadIdx.x] = sm[k] + cc[k];
  __syncthreads();
  if (threadIdx.x < 5) {
    const int k = threadIdx.x;
    double s = 0.0, c = 0.0;
    for (int i = 0; i < (int)blockDim.x; ++i) neumaier3(s, c, red[k][i]);
    partial[5 * (int64_t)blockIdx.x + k] = s + c;
  }
}

hipError_t launch_audit3(const void *buf, const Tile3 *tiles, int ntiles, int64_t plane, int pitch,
                         double *partial, int fp32, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  if (fp32)
    hipLaunchKernelGGL(audit3_kernel<float>, dim3(ntiles), dim3(256), 0, s, static_cast<const float *>(buf),
                       tiles, plane, pitch, partial);
  else
    hipLaunchKernelGGL(audit3_kernel<double>, dim3(ntiles), dim3(256), 0, s, static_cast<const double *>(buf),
                       tiles, plane, pitch, partial);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Rectangle copy-in (f^eq(U) or raw F into both buffers of covered cells) and
// copy-out (W or F of active cells; NaN elsewhere)
// ---------------------------------------------------------------------------
template <class T>
__global__ void set3_kernel(Rect3 a, int raw) {
  const int64_t n = (int64_t)a.nx * a.ny * a.nz;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int x = (int)(i % a.nx), y = (int)((i / a.nx) % a.ny), z = (int)(i / ((int64_t)a.nx * a.ny));
  const int fx = a.x0 + x - a.fx0, fy = a.y0 + y - a.fy0, fz = a.z0 + z - a.fz0;
  const uint8_t st = a.status[((int64_t)fz * a.fh + fy) * a.fw + fx];
  if (st == 0) return;
  const int64_t o = (int64_t)fz * a.slab + (int64_t)fy * a.pitch + fx + a.xoff;
  double f[30];
  if (raw) {
#pragma unroll
    for (int j = 0; j < 30; ++j) f[j] = a.stage[j * n + i];
  } else {
    double W[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) W[k] = a.stage[k * n + i];
    const double rho = W[0], mx = W[1], my = W[2], mz = W[3], E = W[4];
    const double u = mx / rho;
    const double v = my / rho;
    const double w = mz / rho;
    const double p = a.gm1 * (E - 0.5 * ((mx * u + my * v) + mz * w));
    const double Q[3][5] = {{mx, mx * u + p, my * u, mz * u, (E + p) * u},
                            {my, mx * v, my * v + p, mz * v, (E + p) * v},
                            {mz, mx * w, my * w, mz * w + p, (E + p) * w}};
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      const double share = W[k] / 6.0;
#pragma unroll
      for (int al = 0; al < 3; ++al) {
        f[(2 * al) * 5 + k] = share + a.h * Q[al][k];
        f[(2 * al + 1) * 5 + k] = share - a.h * Q[al][k];
      }
    }
  }
  T *b0 = static_cast<T *>(a.buf0), *b1 = static_cast<T *>(a.buf1);
#pragma unroll
  for (int j = 0; j < 30; ++j) {
    b0[j * a.plane + o] = (T)f[j];
    b1[j * a.plane + o] = (T)f[j];
  }
}

template <class T>
__global__ void get3_kernel(Rect3 a, int pops) {
  const int64_t n = (int64_t)a.nx * a.ny * a.nz;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int x = (int)(i % a.nx), y = (int)((i / a.nx) % a.ny), z = (int)(i / ((int64_t)a.nx * a.ny));
  const int fx = a.x0 + x - a.fx0, fy = a.y0 + y - a.fy0, fz = a.z0 + z - a.fz0;
  const bool act = a.status[((int64_t)fz * a.fh + fy) * a.fw + fx] == 1;
  const int64_t o = (int64_t)fz * a.slab + (int64_t)fy * a.pitch + fx + a.xoff;
  const T *b = static_cast<const T *>(a.buf0);
  auto f = [&](int q, int k) { return (double)b[(q * 5 + k) * a.plane + o]; };
  if (pops) {
    for (int j = 0; j < 30; ++j) a.stage[j * n + i] = act ? (double)b[j * a.plane + o] : __builtin_nan("");
  } else {
#pragma unroll
    for (int k = 0; k < 5; ++k)
      a.stage[k * n + i] =
          act ? ((((f(0, k) + f(1, k)) + f(2, k)) + f(3, k)) + f(4, k)) + f(5, k) : __builtin_nan("");
  }
}

hipError_t launch_set3(const Rect3 &a, int raw, int fp32, hipStream_t s) {
  const int64_t n = (int64_t)a.nx * a.ny * a.nz;
  if (n <= 0) return hipSuccess;
  const dim3 grid((unsigned)((n + 255) / 256));
  if (fp32)
    hipLaunchKernelGGL(set3_kernel<float>, grid, dim3(256), 0, s, a, raw);
  else
    hipLaunchKernelGGL(set3_kernel<double>, grid, dim3(256), 0, s, a, raw);
  return hipGetLastError();
}

hipError_t launch_get3(const Rect3 &a, int pops, int fp32, hipStream_t s) {
  const int64_t n = (int64_t)a.nx * a.ny * a.nz;
  if (n <= 0) return hipSuccess;
  const dim3 grid((unsigned)((n + 255) / 256));
  if (fp32)
    hipLaunchKernelGGL(get3_kernel<float>, grid, dim3(256), 0, s, a, pops);
  else
    hipLaunchKernelGGL(get3_kernel<double>, grid, dim3(256), 0, s, a, pops);
  return hipGetLastError();
}

}  // namespace vlbm3

namespace vlbm3 {

// ---------------------------------------------------------------------------
// Regrid (Sec. 3.4 with D = 3): merge r^3 children into their parent (both
// time levels), copy surviving cells into new frames, split a parent into r^3
// children with one minmod slope per axis (both time levels).
// ---------------------------------------------------------------------------
template <class T>
__global__ void merge3_kernel(RegridArgs3 a) {
  const int op = blockIdx.x;
  if (op >= a.nops) return;
  const RegridOp3 o = a.ops[op];
  const T *F = static_cast<const T *>(a.fine_cur);
  T *C0 = static_cast<T *>(a.coarse0), *C1 = static_cast<T *>(a.coarse1);
  const int r = a.r;
  const double rrr = (double)(r * r * r);
  for (int i = threadIdx.x; i < 30; i += blockDim.x) {
    const T *f = F + i * a.fplane + o.src;
    double sum = 0.0;
    for (int g = 0; g < r; ++g)
      for (int b = 0; b < r; ++b)
        for (int x = 0; x < r; ++x) sum += (double)f[(int64_t)g * a.fslab + (int64_t)b * a.fpitch + x];
    const T m = (T)(sum / rrr);
    C0[i * a.cplane + o.dst] = m;
    C1[i * a.cplane + o.dst] = m;
  }
}

template <class T>
__global__ void split3_kernel(RegridArgs3 a) {
  const int op = blockIdx.x;
  if (op >= a.nops) return;
  const RegridOp3 o = a.ops[op];
  const T *C = static_cast<const T *>(a.coarse_cur);
  T *F0 = static_cast<T *>(a.fine0), *F1 = static_cast<T *>(a.fine1);
  const int r = a.r;
  for (int i = threadIdx.x; i < 30; i += blockDim.x) {
    const T *c = C + i * a.cplane;
    const double fi = (double)c[o.src];
    double sl[3];
    for (int ax = 0; ax < 3; ++ax)
      sl[ax] = (o.nb[2 * ax] >= 0 && o.nb[2 * ax + 1] >= 0)
                   ? minmod3(fi - (double)c[o.nb[2 * ax + 1]], (double)c[o.nb[2 * ax]] - fi)
                   : 0.0;
    for (int g = 0; g < r; ++g)
      for (int b = 0; b < r; ++b)
        for (int x = 0; x < r; ++x) {
          const double xa = (double)(2 * x - r + 1) / (double)(2 * r);
          const double xb = (double)(2 * b - r + 1) / (double)(2 * r);
          const double xg = (double)(2 * g - r + 1) / (double)(2 * r);
          double v = fi + sl[0] * xa;
          v = v + sl[1] * xb;
          v = v + sl[2] * xg;
          const int64_t e = i * a.fplane + o.dst + (int64_t)g * a.fslab + (int64_t)b * a.fpitch + x;
          F0[e] = (T)v;
          F1[e] = (T)v;
        }
  }
}

// runs[k] = (src, dst, len): copy len consecutive elements of every plane of
// both buffers from the old frame to the new one.
template <class T>
__global__ void copy3_runs_kernel(const void *s0, const void *s1, void *d0, void *d1, const int32_t *runs,
                                  int nruns, int64_t splane, int64_t dplane) {
  const int k = blockIdx.x;
  if (k >= nruns) return;
  const int32_t src = runs[3 * k], dst = runs[3 * k + 1], len = runs[3 * k + 2];
  const T *a0 = static_cast<const T *>(s0), *a1 = static_cast<const T *>(s1);
  T *b0 = static_cast<T *>(d0), *b1 = static_cast<T *>(d1);
  for (int64_t t = threadIdx.x; t < (int64_t)30 * len; t += blockDim.x) {
    const int i = (int)(t / len), x = (int)(t - (int64_t)i * len);
    b0[i * dplane + dst + x] = a0[i * splane + src + x];
    b1[i * dplane + dst + x] = a1[i * splane + src + x];
  }
}

hipError_t launch_merge3(const RegridArgs3 &a, int fp32, hipStream_t s) {
  if (a.nops <= 0) return hipSuccess;
  if (fp32)
    hipLaunchKernelGGL(merge3_kernel<float>, dim3(a.nops), dim3(64), 0, s, a);
  else
    hipLaunchKernelGGL(merge3_kernel<double>, dim3(a.nops), dim3(64), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_split3(const RegridArgs3 &a, int fp32, hipStream_t s) {
  if (a.nops <= 0) return hipSuccess;
  if (fp32)
    hipLaunchKernelGGL(split3_kernel<float>, dim3(a.nops), dim3(64), 0, s, a);
  else
    hipLaunchKernelGGL(split3_kernel<double>, dim3(a.nops), dim3(64), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_copy3_runs(const void *s0, const void *s1, void *d0, void *d1, const int32_t *runs,
                             int nruns, int64_t splane, int64_t dplane, int fp32, hipStream_t s) {
  if (nruns <= 0) return hipSuccess;
  if (fp32)
    hipLaunchKernelGGL(copy3_runs_kernel<float>, dim3(nruns), dim3(256), 0, s, s0, s1, d0, d1, runs, nruns,
                       splane, dplane);
  else
    hipLaunchKernelGGL(copy3_runs_kernel<double>, dim3(nruns), dim3(256), 0, s, s0, s1, d0, d1, runs, nruns,
                       splane, dplane);
  return hipGetLastError();
}

// Interfaces a regrid creates: population q (5 planes) of each listed ring
// cell gets its current value in the other buffer too (items[2i] element
// offset, items[2i+1] q), so the first hand-off across that face is flat.
template <class T>
__global__ void restart_faces3_kernel(const T *__restrict__ cur, T *__restrict__ other,
                                      const int32_t *items, int n, int64_t P) {
  const int64_t total = (int64_t)n * 5;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = t / 5;
    const int k = (int)(t - i * 5);
    const int64_t e = (int64_t)(items[2 * i + 1] * 5 + k) * P + items[2 * i];
    other[e] = cur[e];
  }
}

hipError_t launch_restart_faces3(const void *cur, void *other, const int32_t *items, int n, int64_t plane,
                                 int fp32, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t total = (int64_t)n * 5;
  const dim3 grid((unsigned)std::min<int64_t>((total + 255) / 256, 65536));
  if (fp32)
    hipLaunchKernelGGL(restart_faces3_kernel<float>, grid, dim3(256), 0, s, static_cast<const float *>(cur),
                       static_cast<float *>(other), items, n, plane);
  else
    hipLaunchKernelGGL(restart_faces3_kernel<double>, grid, dim3(256), 0, s, static_cast<const double *>(cur),
                       static_cast<double *>(other), items, n, plane);
  return hipGetLastError();
}

}  // namespace vlbm3
