// Forward reprojection launchers: the FP32 tiled path (kernels in
// tile_kernels.hpp: FP64 anchors, FP32 per-pixel offsets, LDS-staged source
// boxes) and the two FP64 comparison forms (composed projective map;
// explicit two-stage trigonometry of the paper's section 3.2).
#include "tile_kernels.hpp"

namespace dfr {

using TileKernel = void (*)(FramePlan, TileGeom);

static TileKernel pick_tile_kernel(int interp, int np, int sord) {
  const void *k = interp == DFR_NEAREST    ? tile_kernel_for<DFR_NEAREST>(np, sord)
                  : interp == DFR_BILINEAR ? tile_kernel_for<DFR_BILINEAR>(np, sord)
                                           : tile_kernel_for<DFR_BICUBIC>(np, sord);
  return reinterpret_cast<TileKernel>(const_cast<void *>(k));
}

hipError_t launch_forward_f32(const FramePlan &P, const TileGeom &G, int interp, int np,
                              hipStream_t stream) {
  if (G.n_tiles <= 0) return hipSuccess;
  // a target with SIP A/B needs the kernel that compiles the target SIP in
  TileKernel k = pick_tile_kernel(interp, np, P.t_order > 0 ? kRtOrder : P.s_order);
  size_t lds = (size_t)G.lds_cap * sizeof(float);
  hipLaunchKernelGGL(k, dim3(G.n_tiles), dim3(kThreads), lds, stream, P, G);
  return hipGetLastError();
}

// ------------------------------------------------------ cell models

// One lane per 32x32 cell of the output grid: the certified cubic model of
// the cell's position map (cell_model.hpp), written to the model table.
template <int SORD>
__global__ __launch_bounds__(64) void cell_models_kernel(FramePlan P, int ncx, int n,
                                                        CellModel *__restrict__ out) {
  const int i = blockIdx.x * 64 + threadIdx.x;
  if (i >= n) return;
  const int cy = i / ncx, cx = i - cy * ncx;
  CellModel M;
  cell_model<SORD>(P, cx, cy, M);
  out[i] = M;
}

// The same for every frame of a batch: lane i models cell i % ncells of
// frame i / ncells into out[i] (the frame's table starts at frame * ncells).
template <int SORD>
__global__ __launch_bounds__(64) void cell_models_batch_kernel(const FramePlan *__restrict__ plans,
                                                              int ncx, int ncells, int64_t total,
                                                              CellModel *__restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * 64 + threadIdx.x;
  const bool active = i < total;
  const int frame = active ? (int)(i / ncells) : 0;
  const int c = (int)(i - (int64_t)frame * ncells);
  const int cy = c / ncx, cx = c - cy * ncx;
  // the frame table is read-only here: scalar loads through the constant
  // address space
  using ConstPlan = const __attribute__((address_space(4))) FramePlan;
  ConstPlan *cp = (ConstPlan *)(plans + frame);
  const FramePlan &P = *(const FramePlan *)cp;
  int reach = 0;
  if (active) {
    CellModel M;
    cell_model<SORD>(P, cx, cy, M);
    out[i] = M;
    // can any pixel of the cell have a tap inside the source?  From the
    // model's range over the whole cell, grown by 4 px (more than any tap
    // support and the tile kernel's guard); without a model, the anchor's
    // rigorous test with the widest support
    reach = 1;
    if (P.src_w <= 0 || P.src_h <= 0) {
      reach = 0;
    } else if (!M.certified) {
      Anchor A;
      compute_anchor<SORD, false>(P, cx * kCell, cy * kCell, 4, A);
      reach = A.touch;
    } else {
      const float h = (float)kHalfCell;
      const float rx = (fabsf(M.mx[4]) + fabsf(M.mx[1])) * h + M.ex + 4.0f;
      const float ry = (fabsf(M.my[4]) + fabsf(M.my[1])) * h + M.ey + 4.0f;
      const float xc = (float)M.bx + M.mx[0], yc = (float)M.by + M.my[0];
      reach = (xc + rx >= 0.0f && xc - rx <= (float)(P.src_w - 1) && yc + ry >= 0.0f &&
               yc - ry <= (float)(P.src_h - 1)) ? 1 : 0;
    }
  }
  if (P.reach == nullptr) return;
  // the wave's reaching cells merged first (usually all of one frame)
  int v0 = reach ? kReachBig - cx : 0, v1 = reach ? cx + 1 : 0;
  int v2 = reach ? kReachBig - cy : 0, v3 = reach ? cy + 1 : 0;
  const int f0 = __builtin_amdgcn_readfirstlane(frame);
  const bool one_frame = __ballot(frame != f0) == 0ull;
  if (one_frame) {
    v0 = wave_max(v0);
    v1 = wave_max(v1);
    v2 = wave_max(v2);
    v3 = wave_max(v3);
    if (threadIdx.x == 0 && v1 > 0) {
      atomicMax(P.reach + 0, v0);
      atomicMax(P.reach + 1, v1);
      atomicMax(P.reach + 2, v2);
      atomicMax(P.reach + 3, v3);
    }
  } else if (reach) {
    atomicMax(P.reach + 0, v0);
    atomicMax(P.reach + 1, v1);
    atomicMax(P.reach + 2, v2);
    atomicMax(P.reach + 3, v3);
  }
}

const void *cell_models_batch_ptr(int sord) {
  switch (sord) {
    case 0: return reinterpret_cast<const void *>(cell_models_batch_kernel<0>);
    case 1: return reinterpret_cast<const void *>(cell_models_batch_kernel<1>);
    case 2: return reinterpret_cast<const void *>(cell_models_batch_kernel<2>);
    case 3: return reinterpret_cast<const void *>(cell_models_batch_kernel<3>);
    case 4: return reinterpret_cast<const void *>(cell_models_batch_kernel<4>);
    case 5: return reinterpret_cast<const void *>(cell_models_batch_kernel<5>);
    default: return reinterpret_cast<const void *>(cell_models_batch_kernel<-1>);
  }
}

hipError_t launch_cell_models(const FramePlan &P, int ncx, int ncy, CellModel *out,
                              hipStream_t stream) {
  const int n = ncx * ncy;
  if (n <= 0) return hipSuccess;
  const dim3 grid((n + 63) / 64), block(64);
  switch (P.s_order) {
    case 0: hipLaunchKernelGGL(cell_models_kernel<0>, grid, block, 0, stream, P, ncx, n, out); break;
    case 1: hipLaunchKernelGGL(cell_models_kernel<1>, grid, block, 0, stream, P, ncx, n, out); break;
    case 2: hipLaunchKernelGGL(cell_models_kernel<2>, grid, block, 0, stream, P, ncx, n, out); break;
    case 3: hipLaunchKernelGGL(cell_models_kernel<3>, grid, block, 0, stream, P, ncx, n, out); break;
    case 4: hipLaunchKernelGGL(cell_models_kernel<4>, grid, block, 0, stream, P, ncx, n, out); break;
    case 5: hipLaunchKernelGGL(cell_models_kernel<5>, grid, block, 0, stream, P, ncx, n, out); break;
    default: hipLaunchKernelGGL(cell_models_kernel<-1>, grid, block, 0, stream, P, ncx, n, out); break;
  }
  return hipGetLastError();
}

// ------------------------------------------------------ FP64 comparison forms

// FP64 interpolation at (xs, ys) with zero padding; same rules as the FP32
// path (interior footprint exactly 1, out = S/F where F > 0).
template <int INTERP>
__device__ __forceinline__ void interp_f64(const FramePlan &P, double xs, double ys, double a,
                                           double &out, double &fp) {
  const int W = P.src_w, H = P.src_h;
  auto val = [&](int64_t i, int64_t j) -> double {
    return (double)P.src[j * P.pitch + i];
  };
  if constexpr (INTERP == DFR_NEAREST) {
    double fi = rint(xs), fj = rint(ys);
    bool in = fi >= 0.0 && fi < W && fj >= 0.0 && fj < H;
    out = in ? val((int64_t)fi, (int64_t)fj) : 0.0;
    fp = in ? 1.0 : 0.0;
  } else {
    double fx = floor(xs), fy = floor(ys);
    double t = xs - fx, s = ys - fy;
    int n = INTERP == DFR_BILINEAR ? 2 : 4;
    int64_t i0 = (int64_t)fx - (INTERP == DFR_BICUBIC ? 1 : 0);
    int64_t j0 = (int64_t)fy - (INTERP == DFR_BICUBIC ? 1 : 0);
    double wx[4], wy[4];
    if constexpr (INTERP == DFR_BILINEAR) {
      wx[0] = 1.0 - t; wx[1] = t; wy[0] = 1.0 - s; wy[1] = s;
      wx[2] = wx[3] = wy[2] = wy[3] = 0.0;
    } else {
      double u = 1.0 - t, v = 1.0 - s;
      wx[0] = a * t * u * u;
      wx[1] = fma(fma(a + 2.0, t, -(a + 3.0)), t * t, 1.0);
      wx[2] = fma(fma(a + 2.0, u, -(a + 3.0)), u * u, 1.0);
      wx[3] = a * t * t * u;
      wy[0] = a * s * v * v;
      wy[1] = fma(fma(a + 2.0, s, -(a + 3.0)), s * s, 1.0);
      wy[2] = fma(fma(a + 2.0, v, -(a + 3.0)), v * v, 1.0);
      wy[3] = a * s * s * v;
    }
    double S = 0.0, Fx = 0.0, Fy = 0.0;
    bool all_in = true;
    for (int k = 0; k < n; ++k) {
      bool ix = i0 + k >= 0 && i0 + k < W, iy = j0 + k >= 0 && j0 + k < H;
      all_in = all_in && ix && iy;
      Fx += ix ? wx[k] : 0.0;
      Fy += iy ? wy[k] : 0.0;
    }
    for (int l = 0; l < n; ++l) {
      if (j0 + l < 0 || j0 + l >= H) continue;
      double row = 0.0;
      for (int k = 0; k < n; ++k)
        if (i0 + k >= 0 && i0 + k < W) row = fma(wx[k], val(i0 + k, j0 + l), row);
      S = fma(wy[l], row, S);
    }
    double F = all_in ? 1.0 : Fx * Fy;
    out = all_in ? S : (F > 0.0 ? S / F : 0.0);
    fp = F > 0.0 ? F : 0.0;
  }
}

// Paper section 3.2 literally (trigonometric two-stage form, FP64), with
// the arcsines evaluated as atan2 of the same unit vector.
__device__ __forceinline__ bool position_trig(const FramePlan &P, const TrigPlan &T, double x,
                                              double y, double &xs, double &ys) {
  const double R0 = 57.295779513082320876798;  // 180 / pi
  double u = x - P.tcr[0], v = y - P.tcr[1];
  if (P.t_order > 0) {
    double du = sip_f64_dev(P.tA, P.t_order, u, v);
    double dv = sip_f64_dev(P.tB, P.t_order, u, v);
    u += du;
    v += dv;
  }
  double up = T.tcd[0] * u + T.tcd[1] * v;
  double vp = T.tcd[2] * u + T.tcd[3] * v;
  double r = hypot(up, vp);
  double phi = atan2(-up, vp);
  double theta = atan2(R0, r);
  double st, ct, sp, cp, sd0, cd0;
  sincos(theta, &st, &ct);
  sincos(phi, &sp, &cp);
  sincos(T.tcrval[1], &sd0, &cd0);
  double Z = st * sd0 + ct * cd0 * cp;
  double X = -ct * sp;
  double Y = st * cd0 - ct * sd0 * cp;
  double dec = atan2(Z, hypot(X, Y));
  double ra = T.tcrval[0] + atan2(X, Y);
  // to the source plane
  double sde, cde, sdr, cdr, ss0, cs0;
  sincos(dec, &sde, &cde);
  sincos(ra - T.scrval[0], &sdr, &cdr);
  sincos(T.scrval[1], &ss0, &cs0);
  double X2 = -cde * sdr;
  double Y2 = sde * cs0 - cde * ss0 * cdr;
  double Z2 = sde * ss0 + cde * cs0 * cdr;
  if (!(Z2 > 0.0)) return false;
  double phi2 = atan2(X2, Y2);
  double theta2 = atan2(Z2, hypot(X2, Y2));
  double st2, ct2, sp2, cp2;
  sincos(theta2, &st2, &ct2);
  sincos(phi2, &sp2, &cp2);
  double r2 = R0 * ct2 / st2;
  double xp = -r2 * sp2, yp = r2 * cp2;
  double U = T.scdi[0] * xp + T.scdi[1] * yp;
  double V = T.scdi[2] * xp + T.scdi[3] * yp;
  if (P.s_order > 0) {
    double dU = sip_f64_dev(P.sA, P.s_order, U, V);
    double dV = sip_f64_dev(P.sB, P.s_order, U, V);
    U += dU;
    V += dV;
  }
  xs = U + P.scr[0];
  ys = V + P.scr[1];
  return isfinite(xs) && isfinite(ys);
}

template <int INTERP, bool TRIG>
__global__ __launch_bounds__(kThreads) void reproject_f64(FramePlan P, TrigPlan T, TileGeom G) {
  const int64_t n = (int64_t)G.out_h * G.out_w;
  const float miss = G.nan_outside ? __builtin_nanf("") : 0.0f;
  for (int64_t idx = (int64_t)blockIdx.x * kThreads + threadIdx.x; idx < n;
       idx += (int64_t)gridDim.x * kThreads) {
    const int y = (int)(idx / G.out_w), x = (int)(idx - (int64_t)y * G.out_w);
    double xs = 0.0, ys = 0.0;
    bool ok = TRIG ? position_trig(P, T, x, y, xs, ys) : position_f64_ct<kRtOrder, true>(P, x, y, xs, ys);
    ok = ok && fabs(xs) < 4.0e15 && fabs(ys) < 4.0e15;
    double o = 0.0, f = 0.0;
    if (ok && P.src_h > 0 && P.src_w > 0) interp_f64<INTERP>(P, xs, ys, (double)G.cubic_a, o, f);
    bool cov = f > 0.0;
    P.out[idx] = cov ? (float)o : miss;
    if (P.fp) P.fp[idx] = cov ? (float)f : 0.0f;
    if (G.debug) {
      double2 d;
      d.x = ok ? xs : __builtin_nan("");
      d.y = ok ? ys : __builtin_nan("");
      reinterpret_cast<double2 *>(G.debug)[idx] = d;
    }
  }
}

hipError_t launch_forward_f64(const FramePlan &P, const TrigPlan &T, const TileGeom &G,
                              int interp, bool trig, hipStream_t stream) {
  int64_t n = (int64_t)G.out_h * G.out_w;
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + kThreads - 1) / kThreads;
  if (blocks > 65536 * 8) blocks = 65536 * 8;
  void (*k)(FramePlan, TrigPlan, TileGeom);
  if (trig) {
    k = interp == DFR_NEAREST ? reproject_f64<DFR_NEAREST, true>
        : interp == DFR_BILINEAR ? reproject_f64<DFR_BILINEAR, true>
                                 : reproject_f64<DFR_BICUBIC, true>;
  } else {
    k = interp == DFR_NEAREST ? reproject_f64<DFR_NEAREST, false>
        : interp == DFR_BILINEAR ? reproject_f64<DFR_BILINEAR, false>
                                 : reproject_f64<DFR_BICUBIC, false>;
  }
  hipLaunchKernelGGL(k, dim3((unsigned)blocks), dim3(kThreads), 0, stream, P, T, G);
  return hipGetLastError();
}

// ------------------------------------------------------------ small kernels

__global__ void zero_i32_kernel(int *p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0;
}

const void *zero_i32_kernel_ptr() { return reinterpret_cast<const void *>(zero_i32_kernel); }

hipError_t launch_zero_i32(int *p, int64_t n, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 1024) blocks = 1024;
  hipLaunchKernelGGL(zero_i32_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, p, n);
  return hipGetLastError();
}

}  // namespace dfr
