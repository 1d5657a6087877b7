// dm_segment.h -- closest points of two segments (device code shared by the contact
// detection of dm_contact.hip and the self-contact terms of the step kernel).
//
// Segments p1 + s d1 and p2 + t d2, s, t in [0, 1]: the clamped closest-point construction
// (Ericson, Real-Time Collision Detection, 5.1.9): s minimises the line-line distance,
// clamped to [0, 1]; t follows from s; when t leaves [0, 1] it is clamped and s recomputed
// and clamped.  Parallel segments (or a degenerate d1) take s = 0, one of the equally close
// pairs of points.  Returns |P - Q|^2; r receives P - Q.
#pragma once

__device__ __forceinline__ double seg_dot(const double (&a)[3], const double (&b)[3]) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

__device__ __forceinline__ double seg_clamp01(double v) { return fmin(fmax(v, 0.0), 1.0); }

__device__ inline double seg_closest(const double (&p1)[3], const double (&d1)[3], const double (&p2)[3],
                                     const double (&d2)[3], double& s, double& t, double (&r)[3]) {
  double w[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) w[c] = p1[c] - p2[c];
  const double a = seg_dot(d1, d1), e = seg_dot(d2, d2), f = seg_dot(d2, w);
  const double c0 = seg_dot(d1, w), b = seg_dot(d1, d2);
  const double den = a * e - b * b;
  s = den > 1e-14 * a * e ? seg_clamp01((b * f - c0 * e) / den) : 0.0;
  t = (b * s + f) / e;
  if (t < 0.0) {
    t = 0.0;
    s = seg_clamp01(-c0 / a);
  } else if (t > 1.0) {
    t = 1.0;
    s = seg_clamp01((b - c0) / a);
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) r[c] = fma(s, d1[c], p1[c]) - fma(t, d2[c], p2[c]);
  return seg_dot(r, r);
}
