// Level-1 (Shichman-Hodges) MOSFET evaluation on the device, shared by the
// transient kernels.
#pragma once

#include <hip/hip_runtime.h>

namespace expri {

// ---------------------------------------------------------------------------
// level-1 MOSFET (Shichman-Hodges with channel-length modulation)
// I is the current into the drain terminal; derivatives w.r.t. V_d, V_g, V_s.
// ---------------------------------------------------------------------------

__device__ __forceinline__ void mos_forward(double va, double vg, double vb, double K, double vth,
                                            double lam, double &f, double &fa, double &fg,
                                            double &fb) {
  const double vov = vg - vb - vth;
  const double vds = va - vb;
  f = 0.0; fa = 0.0; fg = 0.0; fb = 0.0;
  if (vov > 0.0) {
    const double q = 1.0 + lam * vds;
    double f_ov, f_ds;
    if (vds < vov) {
      const double P = vov * vds - 0.5 * vds * vds;
      f = K * P * q;
      f_ov = K * vds * q;
      f_ds = K * ((vov - vds) * q + P * lam);
    } else {
      f = 0.5 * K * vov * vov * q;
      f_ov = K * vov * q;
      f_ds = 0.5 * K * vov * vov * lam;
    }
    fa = f_ds;
    fg = f_ov;
    fb = -f_ov - f_ds;
  }
}

__device__ __forceinline__ void mos_eval(double type, double vd, double vg, double vs, double K,
                                         double vth, double lam, double &I, double &dd,
                                         double &dg, double &ds) {
  const double sg = type > 0.0 ? 1.0 : -1.0;   // PMOS = mirror image of NMOS
  vd *= sg; vg *= sg; vs *= sg;
  double f, fa, fg, fb;
  if (vd >= vs) {
    mos_forward(vd, vg, vs, K, vth, lam, f, fa, fg, fb);
    I = f; dd = fa; dg = fg; ds = fb;
  } else {
    mos_forward(vs, vg, vd, K, vth, lam, f, fa, fg, fb);
    I = -f; dd = -fb; dg = -fg; ds = -fa;
  }
  I *= sg;
}

}  // namespace expri
