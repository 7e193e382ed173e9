/*
 * radar_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, brute-force CPU implementation of the rotating-radar scan of
 * RadaRays (Mock, Magnusson, Hertzberg, "RadaRays: Real-time Simulation of
 * Rotating FMCW Radar for Mobile Robotics via Hardware-accelerated Ray
 * Tracing", Sec. III).  It exists to check the HIP library against; only the
 * tests, the smoke check and the benchmark's CPU-baseline leg may load it.
 * It shares no code, header or table with the library.
 *
 * Every segment tests every triangle (no acceleration structure).  Quantities
 * that decide a discrete outcome -- which triangle is hit, in which range bin
 * a return lands, total internal reflection, child directions and origins --
 * are computed in float32 in one fixed operation order (no FMA contraction),
 * the precision of the GPU kernel.  Energies and the image are computed and
 * summed in float64.  Primary directions are computed in float64 and rounded
 * to float32.
 *
 * Pins (see tests/test_oracle_pins.py): Philox against numpy's Philox,
 * erfinv against scipy, the lobe integral against the Gamma closed form,
 * Fresnel/Snell closed forms, a plane at a known distance, a slab, an empty
 * room, energy conservation, mirror and rotation symmetry.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

#pragma STDC FP_CONTRACT OFF

#define ORC_BEAM_GAIN 1u
#define ORC_FIXED_PATTERN 2u
#define ORC_MIRROR_PAIRS 4u
#define ORC_RETURN_ALL 8u
#define ORC_AIR_PATH 16u

#define ORC_DIELECTRIC 0u
#define ORC_METAL 1u
#define ORC_LAMBERTIAN 2u
#define ORC_COOK_TORRANCE 3u

typedef struct {
  float position[3];
  float quat_wxyz[4];
} orc_pose;

typedef struct {
  uint32_t n_azimuth, rays_per_beam, max_bounces, n_bins;
  float bin_size_m, beam_width_rad, beam_prob, energy_cutoff;
  uint64_t seed;
  uint32_t scan_id, flags;
  float stretch_az, stretch_inc; /* elliptic beam: scale of the cone offsets (0 = 1) */
} orc_params;

typedef struct {
  uint32_t kind;
  float n, reflectance, A, B, C;
} orc_material;

/* energy bookkeeping slots, per column */
enum { E_EMITTED = 0, E_RET_IN, E_RET_OUT, E_ESCAPED, E_ABSORBED, E_TERMINATED, E_CUT, E_BLOCKED, E_NSLOTS };

/* ------------------------------------------------------------------------ */
/* Philox4x64-10 counter-based generator (Salmon, Moraes, Dror, Shaw,        */
/* "Parallel random numbers: as easy as 1, 2, 3", SC'11).                    */
/* ------------------------------------------------------------------------ */
static const uint64_t PHILOX_M0 = 0xD2E7470EE14C6C93ull;
static const uint64_t PHILOX_M1 = 0xCA5A826395121157ull;
static const uint64_t PHILOX_W0 = 0x9E3779B97F4A7C15ull;
static const uint64_t PHILOX_W1 = 0xBB67AE8584CAA73Bull;

void orc_philox4x64_10(const uint64_t key[2], const uint64_t ctr[4], uint64_t out[4]) {
  uint64_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
  uint64_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += PHILOX_W0;
      k1 += PHILOX_W1;
    }
    unsigned __int128 p0 = (unsigned __int128)PHILOX_M0 * x0;
    unsigned __int128 p1 = (unsigned __int128)PHILOX_M1 * x2;
    uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
    uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
    uint64_t y0 = hi1 ^ x1 ^ k0, y2 = hi0 ^ x3 ^ k1;
    x0 = y0;
    x1 = lo1;
    x2 = y2;
    x3 = lo0;
  }
  out[0] = x0;
  out[1] = x1;
  out[2] = x2;
  out[3] = x3;
}

/* ------------------------------------------------------------------------ */
/* Beam-cone radius scale of the D3 density (Sec. III-A, Eq. 2):            */
/*   r = N(0,1) * (b/2) / (sqrt(2) * erfinv(P))                              */
/* erfinv by bisection on the C library's erf.                               */
/* ------------------------------------------------------------------------ */
double orc_erfinv(double p) {
  if (!(p > -1.0 && p < 1.0)) return NAN;
  /* erfinv is odd; for |p| > 1/2 bisect on erfc(x) = 1 - |p|, which keeps
   * the resolution that erf loses near 1 */
  double ap = fabs(p), q = 1.0 - ap;
  double lo = 0.0, hi = 7.0;
  for (int i = 0; i < 400; ++i) {
    double mid = 0.5 * (lo + hi);
    if (mid == lo || mid == hi) break;
    int below = ap <= 0.5 ? (erf(mid) < ap) : (erfc(mid) > q);
    if (below)
      lo = mid;
    else
      hi = mid;
  }
  double x = 0.5 * (lo + hi);
  return p < 0.0 ? -x : x;
}

double orc_sigma_r(double beam_width, double beam_prob) {
  return (beam_width / 2.0) / (sqrt(2.0) * orc_erfinv(beam_prob));
}

/* ------------------------------------------------------------------------ */
/* Standard BRDF (Sec. III-A, Eq. 5) as the shape of the reflected energy   */
/* density; normalised so it integrates to one over [-pi/2, pi/2] (Eq. 3)   */
/* and integrated over a beam window of width b (Eq. 4).                     */
/* ------------------------------------------------------------------------ */
/* integrand of I(C) on [0, pi/2] after alpha = (pi/2)(1 - (1-x)^4): smooth
 * at the end point alpha = pi/2 for every C >= 0 */
static double lobe_graded(double C, double x) {
  double y = 1.0 - x, y3 = y * y * y;
  double alpha = (M_PI / 2.0) * (1.0 - y3 * y);
  return pow(cos(alpha), C) * (M_PI / 2.0) * 4.0 * y3;
}

/* I(C) = integral over [-pi/2, pi/2] of cos(alpha)^C, composite Simpson. */
double orc_lobe_integral(double C) {
  if (C == 0.0) return M_PI;
  const int n = 1 << 17;
  double h = 1.0 / n, s = lobe_graded(C, 0.0) + lobe_graded(C, 1.0);
  for (int i = 1; i < n; ++i) s += (i & 1 ? 4.0 : 2.0) * lobe_graded(C, i * h);
  return 2.0 * s * h / 3.0;
}

/* out = {Z, a, beta, s}:  Z = A*pi + 2B + S*I(C);
 * the beam-window return fraction is w(c) = a + beta*c + s*c^C with
 * a = A*b/Z, beta = 2B*sin(b/2)/Z, s = S*b/Z (the S term integrated over the
 * window with the one-point midpoint rule, the A and B terms exactly). */
void orc_window_coeffs(const orc_material* m, double b, double out[4]) {
  if (m->kind == ORC_COOK_TORRANCE) {
    /* a three-dimensional BRDF: the window is the solid angle of the cone
     * of opening angle b around the return direction */
    out[0] = 2.0 * M_PI * (1.0 - cos(b / 2.0));
    out[1] = out[2] = out[3] = 0.0;
    return;
  }
  double A = m->A, B = m->B, S = 1.0 - A - B;
  double Z = A * M_PI + 2.0 * B + S * orc_lobe_integral(m->C);
  out[0] = Z;
  out[1] = A * b / Z;
  out[2] = 2.0 * B * sin(b / 2.0) / Z;
  out[3] = S * b / Z;
}

/* ------------------------------------------------------------------------ */
/* Cook-Torrance microfacet BRDF as a second material kind (the user-defined */
/* BRDF of the experiments, Sec. IV): Cook & Torrance (1982) with the GGX     */
/* normal distribution and the separable Smith masking of Walter et al.      */
/* (2007).  Material fields: A = diffuse amount k_d, B = roughness alpha,    */
/* n = index of refraction of the Fresnel factor, reflectance = reflected    */
/* share (1 - transmittance).  For unit vectors n (surface, towards the      */
/* incoming side), l (towards where the ray came from) and v (return):       */
/*   f = k_d / pi + (1 - k_d) D(h) F(v.h) G1(n.l) G1(n.v) / (4 (n.l)(n.v)),   */
/*   h = (l + v) / |l + v|, D = a^2 / (pi ((n.h)^2 (a^2 - 1) + 1)^2),        */
/*   G1(x) = 2x / (x + sqrt(a^2 + (1 - a^2) x^2)), F the unpolarised         */
/*   Fresnel reflectance from index 1 into n at cos = v.h;                   */
/* out = {D, F, G1(n.l) G1(n.v), f}; f = 0 unless n.l > 0 and n.v > 0.       */
/* ------------------------------------------------------------------------ */
static double fresnel_unpolarised(double N1, double N2, double ci) {
  double e = N1 / N2;
  double k64 = 1.0 - e * e * (1.0 - ci * ci);
  if (k64 < 0.0) return 1.0;
  double ct = sqrt(k64);
  double ds = N1 * ci + N2 * ct, dp = N2 * ci + N1 * ct;
  if (ds == 0.0 || dp == 0.0) return 1.0;
  double rs = (N1 * ci - N2 * ct) / ds;
  double rp = (N2 * ci - N1 * ct) / dp;
  return 0.5 * (rs * rs + rp * rp);
}

void orc_ct_terms(const orc_material* m, const double n[3], const double l[3], const double v[3],
                  double out[4]) {
  out[0] = out[1] = out[2] = out[3] = 0.0;
  double nl = n[0] * l[0] + n[1] * l[1] + n[2] * l[2];
  double nv = n[0] * v[0] + n[1] * v[1] + n[2] * v[2];
  if (!(nl > 0.0 && nv > 0.0)) return;
  double h[3] = {l[0] + v[0], l[1] + v[1], l[2] + v[2]};
  double hl = sqrt(h[0] * h[0] + h[1] * h[1] + h[2] * h[2]);
  h[0] = h[0] / hl;
  h[1] = h[1] / hl;
  h[2] = h[2] / hl;
  double nh = n[0] * h[0] + n[1] * h[1] + n[2] * h[2];
  double vh = v[0] * h[0] + v[1] * h[1] + v[2] * h[2];
  double a = m->B, a2 = a * a;
  double q = nh * nh * (a2 - 1.0) + 1.0;
  double D = a2 / (M_PI * q * q);
  double g1l = 2.0 * nl / (nl + sqrt(a2 + (1.0 - a2) * nl * nl));
  double g1v = 2.0 * nv / (nv + sqrt(a2 + (1.0 - a2) * nv * nv));
  double F = fresnel_unpolarised(1.0, (double)m->n, vh);
  double kd = m->A;
  out[0] = D;
  out[1] = F;
  out[2] = g1l * g1v;
  out[3] = kd / M_PI + (1.0 - kd) * D * F * g1l * g1v / (4.0 * nl * nv);
}

/* share of the reflected energy returned into the beam window around v:
 * f(l, v) (n.v) Omega, clamped to [0, 1] */
static double ct_return(const orc_material* m, const float nf[3], const float d[3], const float v[3],
                        double omega) {
  double n[3] = {nf[0], nf[1], nf[2]}, l[3] = {-(double)d[0], -(double)d[1], -(double)d[2]};
  double vv[3] = {v[0], v[1], v[2]}, t[4];
  orc_ct_terms(m, n, l, vv, t);
  double nv = n[0] * vv[0] + n[1] * vv[1] + n[2] * vv[2];
  double w = t[3] * nv * omega;
  return w < 0.0 ? 0.0 : (w > 1.0 ? 1.0 : w);
}

/* ------------------------------------------------------------------------ */
/* float32 vector helpers, fixed operation order                             */
/* ------------------------------------------------------------------------ */
static inline float dotf(const float a[3], const float b[3]) {
  float xy = a[0] * b[0] + a[1] * b[1];
  return xy + a[2] * b[2];
}
static inline void crossf(const float a[3], const float b[3], float r[3]) {
  r[0] = a[1] * b[2] - a[2] * b[1];
  r[1] = a[2] * b[0] - a[0] * b[2];
  r[2] = a[0] * b[1] - a[1] * b[0];
}
static inline void subf(const float a[3], const float b[3], float r[3]) {
  r[0] = a[0] - b[0];
  r[1] = a[1] - b[1];
  r[2] = a[2] - b[2];
}
static inline void normalizef(float v[3]) {
  float len = sqrtf(dotf(v, v));
  v[0] = v[0] / len;
  v[1] = v[1] / len;
  v[2] = v[2] / len;
}

/* Moller & Trumbore 1997, float32, both faces, inclusive barycentric bounds;
 * accepts 0 < t <= tmax.  e1 = v1 - v0, e2 = v2 - v0. */
static int mt_hit(const float o[3], const float d[3], const float v0[3], const float e1[3],
                  const float e2[3], float tmax, float* t_out) {
  float p[3], s[3], q[3];
  crossf(d, e2, p);
  float det = dotf(e1, p);
  if (det == 0.0f) return 0;
  float inv = 1.0f / det;
  subf(o, v0, s);
  float u = dotf(s, p) * inv;
  if (u < 0.0f || u > 1.0f) return 0;
  crossf(s, e1, q);
  float v = dotf(d, q) * inv;
  if (v < 0.0f || u + v > 1.0f) return 0;
  float t = dotf(e2, q) * inv;
  if (!(t > 0.0f && t <= tmax)) return 0;
  *t_out = t;
  return 1;
}

int orc_ray_triangle(const float o[3], const float d[3], const float v0[3], const float v1[3],
                     const float v2[3], float tmax, float* t) {
  float e1[3], e2[3];
  subf(v1, v0, e1);
  subf(v2, v0, e2);
  return mt_hit(o, d, v0, e1, e2, tmax, t);
}

/* Barycentrics of the hit in float64 (used only to flag near-edge hits). */
static void bary64(const float o[3], const float d[3], const float v0[3], const float e1[3],
                   const float e2[3], double* u_out, double* v_out) {
  double O[3] = {o[0], o[1], o[2]}, D[3] = {d[0], d[1], d[2]};
  double E1[3] = {e1[0], e1[1], e1[2]}, E2[3] = {e2[0], e2[1], e2[2]};
  double P[3] = {D[1] * E2[2] - D[2] * E2[1], D[2] * E2[0] - D[0] * E2[2],
                 D[0] * E2[1] - D[1] * E2[0]};
  double det = E1[0] * P[0] + E1[1] * P[1] + E1[2] * P[2];
  double S[3] = {O[0] - v0[0], O[1] - v0[1], O[2] - v0[2]};
  double Q[3] = {S[1] * E1[2] - S[2] * E1[1], S[2] * E1[0] - S[0] * E1[2],
                 S[0] * E1[1] - S[1] * E1[0]};
  *u_out = (S[0] * P[0] + S[1] * P[1] + S[2] * P[2]) / det;
  *v_out = (D[0] * Q[0] + D[1] * Q[1] + D[2] * Q[2]) / det;
}

/* Origin offset of Waechter & Binder, "A Fast and Robust Method for Avoiding
 * Self-Intersection" (Ray Tracing Gems, 2019, ch. 6): move p along n by a
 * fixed number of float ulps, or by a fixed distance near the origin. */
void orc_offset(const float p[3], const float n[3], float out[3]) {
  const float origin = 1.0f / 32.0f, float_scale = 1.0f / 65536.0f, int_scale = 256.0f;
  for (int i = 0; i < 3; ++i) {
    int32_t of = (int32_t)(int_scale * n[i]);
    int32_t bits;
    memcpy(&bits, &p[i], 4);
    bits += (p[i] < 0.0f) ? -of : of;
    float pi;
    memcpy(&pi, &bits, 4);
    out[i] = fabsf(p[i]) < origin ? p[i] + float_scale * n[i] : pi;
  }
}

/* ------------------------------------------------------------------------ */
/* Primary rays: D3 Gaussian cone (Sec. III-A, Eq. 2) around the azimuth    */
/* k * 2pi / N_az of the rotating sensor (Sec. III-B).                       */
/* ------------------------------------------------------------------------ */
typedef struct {
  double sigma_r;
  double R[3][3];
  float E0;
} prim_consts;

static void make_prim_consts(const orc_params* prm, const orc_pose* pose, prim_consts* pc) {
  pc->sigma_r = orc_sigma_r(prm->beam_width_rad, prm->beam_prob);
  double w = pose->quat_wxyz[0], x = pose->quat_wxyz[1], y = pose->quat_wxyz[2],
         z = pose->quat_wxyz[3];
  double qn = sqrt(w * w + x * x + y * y + z * z);
  w /= qn;
  x /= qn;
  y /= qn;
  z /= qn;
  pc->R[0][0] = 1.0 - 2.0 * (y * y + z * z);
  pc->R[0][1] = 2.0 * (x * y - w * z);
  pc->R[0][2] = 2.0 * (x * z + w * y);
  pc->R[1][0] = 2.0 * (x * y + w * z);
  pc->R[1][1] = 1.0 - 2.0 * (x * x + z * z);
  pc->R[1][2] = 2.0 * (y * z - w * x);
  pc->R[2][0] = 2.0 * (x * z - w * y);
  pc->R[2][1] = 2.0 * (y * z + w * x);
  pc->R[2][2] = 1.0 - 2.0 * (x * x + y * y);
  pc->E0 = 1.0f / (float)prm->rays_per_beam;
}

static void primary(const orc_params* prm, const orc_pose* pose, const prim_consts* pc,
                    uint32_t k, uint32_t i, float o[3], float d[3], float* g, double* z_out,
                    double* omega_out) {
  uint64_t key[2] = {prm->seed, (uint64_t)prm->scan_id};
  uint64_t ck = (prm->flags & ORC_FIXED_PATTERN) ? 0u : k;
  uint64_t ci = (prm->flags & ORC_MIRROR_PAIRS) ? (uint64_t)(i / 2u) : i;
  uint64_t ctr[4] = {ck, ci, 0, 0}, x[4];
  orc_philox4x64_10(key, ctr, x);
  const double two53 = 1.0 / 9007199254740992.0;
  double u1 = (double)((x[0] >> 11) + 1u) * two53; /* (0, 1] */
  double u2 = (double)(x[1] >> 11) * two53;        /* [0, 1) */
  double u3 = (double)(x[2] >> 11) * two53;        /* [0, 1) */
  double zz = sqrt(-2.0 * log(u1)) * cos(2.0 * M_PI * u2); /* Box-Muller */
  double omega = -M_PI + 2.0 * M_PI * u3;
  double r = zz * pc->sigma_r;
  double az_off = r * cos(omega), inc_off = r * sin(omega);
  /* elliptic beam (Sec. III-A): the cone stretched along the two axes */
  if (prm->stretch_az > 0.0f) az_off = az_off * (double)prm->stretch_az;
  if (prm->stretch_inc > 0.0f) inc_off = inc_off * (double)prm->stretch_inc;
  if ((prm->flags & ORC_MIRROR_PAIRS) && (i & 1u)) az_off = -az_off;
  double phi = 2.0 * M_PI * (double)k / (double)prm->n_azimuth + az_off;
  double theta = inc_off;
  double ds[3] = {cos(theta) * cos(phi), cos(theta) * sin(phi), sin(theta)};
  double dw[3];
  for (int a = 0; a < 3; ++a) dw[a] = pc->R[a][0] * ds[0] + pc->R[a][1] * ds[1] + pc->R[a][2] * ds[2];
  double len = sqrt(dw[0] * dw[0] + dw[1] * dw[1] + dw[2] * dw[2]);
  for (int a = 0; a < 3; ++a) {
    d[a] = (float)(dw[a] / len);
    o[a] = pose->position[a];
  }
  *g = (prm->flags & ORC_BEAM_GAIN) ? (float)exp(-0.5 * zz * zz) : 1.0f;
  if (z_out) *z_out = zz;
  if (omega_out) *omega_out = omega;
}

void orc_primary(const orc_params* prm, const orc_pose* pose, uint32_t k, uint32_t i, float o[3],
                 float d[3], float* g, double* z, double* omega) {
  prim_consts pc;
  make_prim_consts(prm, pose, &pc);
  primary(prm, pose, &pc, k, i, o, d, g, z, omega);
}

/* ------------------------------------------------------------------------ */
/* Interaction at a hit (Sec. III-A): Snell, Fresnel, BRDF return, children */
/* ------------------------------------------------------------------------ */
typedef struct {
  int entering, tir, has_refract;
  float nf[3], cosi, kappa, n2, refl_dir[3], refr_dir[3];
  double R, T, w;
} interaction;

static void interact(const float d[3], const float ng[3], const orc_material* m,
                     const double win[4], float n_cur, uint32_t flags, interaction* it) {
  float dn = dotf(d, ng);
  it->entering = dn < 0.0f;
  for (int a = 0; a < 3; ++a) it->nf[a] = it->entering ? ng[a] : -ng[a];
  float dnf = dotf(d, it->nf);
  float cosi = -dnf;
  it->cosi = cosi;
  /* mirror direction: d - 2 (d.n) n */
  float k2 = 2.0f * dnf;
  for (int a = 0; a < 3; ++a) it->refl_dir[a] = d[a] - k2 * it->nf[a];
  normalizef(it->refl_dir);
  it->tir = 0;
  it->has_refract = 0;
  it->kappa = 0.0f;
  it->n2 = n_cur;
  double ci = (double)cosi;
  if (m->kind == ORC_DIELECTRIC || m->kind == ORC_COOK_TORRANCE) {
    float n1 = n_cur, n2 = it->entering ? m->n : 1.0f;
    float eta = n1 / n2;
    float kappa = 1.0f - (eta * eta) * (1.0f - cosi * cosi);
    it->kappa = kappa;
    it->n2 = n2;
    if (kappa < 0.0f) {
      it->tir = 1;
      it->R = 1.0;
      it->T = 0.0;
    } else {
      float cost = sqrtf(kappa);
      float a = eta * cosi - cost;
      for (int c = 0; c < 3; ++c) {
        float ed = eta * d[c];
        it->refr_dir[c] = ed + a * it->nf[c];
      }
      normalizef(it->refr_dir);
      it->has_refract = 1;
      if (m->kind == ORC_COOK_TORRANCE) {
        /* a fixed reflected share; the transmitted rest refracts */
        it->R = m->reflectance;
        it->T = 1.0 - it->R;
        goto returned;
      }
      /* unpolarised Fresnel reflectance, float64 */
      double N1 = n1, N2 = n2;
      double e = N1 / N2;
      double k64 = 1.0 - e * e * (1.0 - ci * ci);
      double ct = sqrt(k64 > 0.0 ? k64 : 0.0);
      double ds = N1 * ci + N2 * ct, dp = N2 * ci + N1 * ct;
      if (ds == 0.0 || dp == 0.0) {
        it->R = 1.0;
      } else {
        double rs = (N1 * ci - N2 * ct) / ds;
        double rp = (N2 * ci - N1 * ct) / dp;
        it->R = 0.5 * (rs * rs + rp * rp);
      }
      it->T = 1.0 - it->R;
    }
  } else {
    it->R = m->reflectance;
    it->T = 0.0;
  }
returned:
  if (flags & ORC_RETURN_ALL) {
    it->w = 1.0;
  } else if (m->kind == ORC_COOK_TORRANCE) {
    /* retrace: the return direction is the way back, -d */
    float back[3] = {-d[0], -d[1], -d[2]};
    it->w = ct_return(m, it->nf, d, back, win[0]);
  } else {
    /* angle between mean reflection and the way back is twice the incidence
     * angle: cos(omega) = 2 cos^2(theta0) - 1, clamped at 0 */
    double c = 2.0 * ci * ci - 1.0;
    if (c < 0.0) c = 0.0;
    double w = win[1] + win[2] * c + win[3] * pow(c, (double)m->C);
    it->w = w < 0.0 ? 0.0 : (w > 1.0 ? 1.0 : w);
  }
}

/* Exposed for the closed-form pins. out_f: {entering, tir, has_refract,
 * cosi, kappa, n2, refl[3], refr[3]}; out_d: {R, T, w}. */
void orc_interact(const float d[3], const float ng[3], const orc_material* m, float beam_width,
                  float n_cur, uint32_t flags, float out_f[12], double out_d[3]) {
  double win[4];
  orc_window_coeffs(m, beam_width, win);
  interaction it;
  interact(d, ng, m, win, n_cur, flags, &it);
  out_f[0] = (float)it.entering;
  out_f[1] = (float)it.tir;
  out_f[2] = (float)it.has_refract;
  out_f[3] = it.cosi;
  out_f[4] = it.kappa;
  out_f[5] = it.n2;
  for (int a = 0; a < 3; ++a) {
    out_f[6 + a] = it.refl_dir[a];
    out_f[9 + a] = it.has_refract ? it.refr_dir[a] : 0.0f;
  }
  out_d[0] = it.R;
  out_d[1] = it.T;
  out_d[2] = it.w;
}

/* ------------------------------------------------------------------------ */
/* The scan                                                                  */
/* ------------------------------------------------------------------------ */
typedef struct {
  /* scene, float32 precomputed per triangle */
  uint32_t nt;
  float *v0, *e1, *e2, *ng; /* [nt][3] */
  uint8_t* degenerate;
  const uint16_t* mat;
  const orc_material* mats;
  double (*win)[4];
  /* scan */
  const orc_params* prm;
  const orc_pose* pose;
  prim_consts pc;
  float r_max;
  uint32_t n_heap;     /* 2^B - 1 */
  uint32_t rec_stride; /* records per primary: n_heap, twice that with air-path returns */
  /* columns */
  const uint32_t* columns;
  uint32_t n_columns;
  const uint8_t* primary_mask;
  /* outputs */
  double* image;
  int32_t* records;
  uint8_t* exempt;
  double* energy;
  uint64_t* seg_per_col;
  /* work distribution */
  uint32_t next_col;
} scan_ctx;

typedef struct {
  float o[3], d[3];
  double E;
  float L, g, n_cur;
  uint32_t depth, heap;
  int32_t excl;
} oray;

typedef struct {
  double* img;      /* column row */
  double* energy;   /* column energy slots */
  int32_t* rec;     /* primary's records or NULL */
  int32_t* air_rec; /* primary's air-path outcomes or NULL */
  double axis[3];   /* the column's beam axis in the world frame */
  int exempt;
  uint64_t segments;
} prim_state;

/* Visibility of the sensor along an air path: does any triangle other than
 * `excl` meet the segment from o along unit s at 0 < t <= dist (the range
 * rule of the closest-hit test)?  Flags the primary when a blocking
 * triangle is hit within 1e-5 of an edge or of the segment's end. */
static int air_blocked(const scan_ctx* c, const float o[3], const float s[3], float dist, int32_t excl,
                       prim_state* ps) {
  int blocked = 0;
  for (uint32_t j = 0; j < c->nt; ++j) {
    if ((int32_t)j == excl || c->degenerate[j]) continue;
    float t;
    if (!mt_hit(o, s, c->v0 + 3 * j, c->e1 + 3 * j, c->e2 + 3 * j, dist, &t)) continue;
    blocked = 1;
    double u, v;
    bary64(o, s, c->v0 + 3 * j, c->e1 + 3 * j, c->e2 + 3 * j, &u, &v);
    double w = 1.0 - u - v;
    double mn = u < v ? u : v;
    mn = mn < w ? mn : w;
    if (!(mn >= 1e-5)) ps->exempt = 1;
    if (fabs((double)t - (double)dist) < 1e-5 * (double)dist) ps->exempt = 1;
  }
  return blocked;
}

static void trace_ray(const scan_ctx* c, const oray* r, prim_state* ps) {
  const orc_params* prm = c->prm;
  ps->segments++;
  float tmax = (c->r_max - r->L) / r->n_cur;
  int32_t best = -1;
  float best_t = 0.0f, second_t = INFINITY;
  for (uint32_t j = 0; j < c->nt; ++j) {
    if ((int32_t)j == r->excl || c->degenerate[j]) continue;
    float t;
    if (!mt_hit(r->o, r->d, c->v0 + 3 * j, c->e1 + 3 * j, c->e2 + 3 * j, tmax, &t)) continue;
    if (best < 0 || t < best_t) {
      if (best >= 0) second_t = best_t;
      best = (int32_t)j;
      best_t = t;
    } else {
      /* equal t keeps the lower index, which was seen first */
      if (t < second_t) second_t = t;
    }
  }
  if (ps->rec) ps->rec[r->heap - 1] = best;
  if (best < 0) {
    ps->energy[E_ESCAPED] += r->E;
    return;
  }
  uint32_t j = (uint32_t)best;
  /* near-edge / near-tie flags (float64) */
  {
    double u, v;
    bary64(r->o, r->d, c->v0 + 3 * j, c->e1 + 3 * j, c->e2 + 3 * j, &u, &v);
    double w = 1.0 - u - v;
    double mn = u < v ? u : v;
    mn = mn < w ? mn : w;
    if (!(mn >= 1e-5)) ps->exempt = 1;
    if (second_t != INFINITY && fabs((double)second_t - (double)best_t) < 1e-5 * (double)best_t)
      ps->exempt = 1;
  }
  const orc_material* m = &c->mats[c->mat[j]];
  interaction it;
  interact(r->d, c->ng + 3 * j, m, c->win[c->mat[j]], r->n_cur, prm->flags, &it);
  if ((m->kind == ORC_DIELECTRIC || m->kind == ORC_COOK_TORRANCE) && fabs((double)it.kappa) < 1e-6) ps->exempt = 1;

  /* return along the travelled path, binned by one-way optical range */
  double e_ret = r->E * it.R * it.w;
  float range = r->L + r->n_cur * best_t;
  float q = range / prm->bin_size_m;
  {
    double qd = (double)range / (double)prm->bin_size_m;
    if (fabs(qd - floor(qd + 0.5)) < 1e-5) ps->exempt = 1;
  }
  if (q < (float)prm->n_bins) {
    uint32_t bin = (uint32_t)q;
    ps->img[bin] += e_ret * (double)r->g;
    ps->energy[E_RET_IN] += e_ret;
  } else {
    ps->energy[E_RET_OUT] += e_ret;
  }
  ps->energy[E_ABSORBED] += r->E * (1.0 - it.R - it.T);

  /* return along the air path (Sec. III-A, multi-path reflection): from a
   * hit at depth >= 1 of a ray travelling in air straight back to the
   * sensor.  Its window angle is the one between the mean reflection and
   * the direction to the sensor; it leaves from the offset origin of the
   * reflected child, needs the sensor on the incoming side of the surface
   * and an unblocked segment, takes the receive gain of its arrival
   * direction and lands at half the round-trip path.  Its energy comes out
   * of the reflected share, at most what the retrace return left. */
  double e_air = 0.0;
  if ((prm->flags & ORC_AIR_PATH) && r->depth >= 1 && r->n_cur == 1.0f) {
    float ph[3], po[3], v[3];
    for (int a = 0; a < 3; ++a) {
      float td = best_t * r->d[a];
      ph[a] = r->o[a] + td;
    }
    orc_offset(ph, it.nf, po);
    for (int a = 0; a < 3; ++a) v[a] = c->pose->position[a] - po[a];
    float dist = sqrtf(dotf(v, v));
    float s[3] = {0.0f, 0.0f, 0.0f};
    if (dist > 0.0f) {
      s[0] = v[0] / dist;
      s[1] = v[1] / dist;
      s[2] = v[2] / dist;
    }
    if (dist > 0.0f && dotf(s, it.nf) > 0.0f) {
      double w_air;
      if (prm->flags & ORC_RETURN_ALL) {
        w_air = 1.0;
      } else if (m->kind == ORC_COOK_TORRANCE) {
        w_air = ct_return(m, it.nf, r->d, s, c->win[c->mat[j]][0]);
      } else {
        double ca = (double)it.refl_dir[0] * s[0] + (double)it.refl_dir[1] * s[1] + (double)it.refl_dir[2] * s[2];
        if (ca < 0.0) ca = 0.0;
        if (ca > 1.0) ca = 1.0;
        const double* wn = c->win[c->mat[j]];
        w_air = wn[1] + wn[2] * ca + wn[3] * pow(ca, (double)m->C);
        w_air = w_air < 0.0 ? 0.0 : (w_air > 1.0 ? 1.0 : w_air);
      }
      e_air = r->E * it.R * w_air;
      double room = r->E * it.R - e_ret;
      if (e_air > room) e_air = room;
      double g_air = 1.0;
      if (prm->flags & ORC_BEAM_GAIN) {
        /* angle between the beam axis and the arrival direction (sensor
         * towards the origin of the return), in float64 from the exact
         * difference of the two float32 points: atan2(|a x w|, a . w) */
        const double* ax = ps->axis;
        double w0 = (double)po[0] - (double)c->pose->position[0];
        double w1 = (double)po[1] - (double)c->pose->position[1];
        double w2 = (double)po[2] - (double)c->pose->position[2];
        double x0 = ax[1] * w2 - ax[2] * w1, x1 = ax[2] * w0 - ax[0] * w2, x2 = ax[0] * w1 - ax[1] * w0;
        double alpha = atan2(sqrt(x0 * x0 + x1 * x1 + x2 * x2), ax[0] * w0 + ax[1] * w1 + ax[2] * w2);
        if (c->pc.sigma_r > 0.0) {
          double z = alpha / c->pc.sigma_r;
          g_air = exp(-0.5 * z * z);
        } else {
          g_air = alpha == 0.0 ? 1.0 : 0.0;
        }
      }
      float range_air = (range + dist) * 0.5f;
      float qa = range_air / prm->bin_size_m;
      {
        double qd = (double)range_air / (double)prm->bin_size_m;
        if (fabs(qd - floor(qd + 0.5)) < 1e-5) ps->exempt = 1;
      }
      int32_t outcome;
      if (qa < (float)prm->n_bins) {
        if (air_blocked(c, po, s, dist, (int32_t)j, ps)) {
          ps->energy[E_BLOCKED] += e_air;
          outcome = 1;
        } else {
          ps->img[(uint32_t)qa] += e_air * g_air;
          ps->energy[E_RET_IN] += e_air;
          outcome = 0;
        }
      } else {
        ps->energy[E_RET_OUT] += e_air;
        outcome = 2;
      }
      if (ps->air_rec) ps->air_rec[r->heap - 1] = outcome;
    }
  }

  double e_refl = r->E * it.R - e_ret - e_air;
  double e_refr = it.has_refract ? r->E * it.T : 0.0;
  if (r->depth + 1 >= prm->max_bounces) {
    ps->energy[E_TERMINATED] += e_refl + e_refr;
    return;
  }
  float p_hit[3];
  for (int a = 0; a < 3; ++a) {
    float td = best_t * r->d[a];
    p_hit[a] = r->o[a] + td;
  }
  double ecut = prm->energy_cutoff;
  /* reflected child */
  if (e_refl > ecut) {
    if (e_refl < 2.0 * ecut) ps->exempt = 1;
    oray ch;
    orc_offset(p_hit, it.nf, ch.o);
    memcpy(ch.d, it.refl_dir, sizeof ch.d);
    ch.E = e_refl;
    ch.L = range;
    ch.g = r->g;
    ch.n_cur = r->n_cur;
    ch.depth = r->depth + 1;
    ch.heap = 2u * r->heap;
    ch.excl = (int32_t)j;
    trace_ray(c, &ch, ps);
  } else {
    if (e_refl > 0.5 * ecut) ps->exempt = 1;
    ps->energy[E_CUT] += e_refl;
  }
  /* refracted child */
  if (it.has_refract) {
    if (e_refr > ecut) {
      if (e_refr < 2.0 * ecut) ps->exempt = 1;
      oray ch;
      float neg[3] = {-it.nf[0], -it.nf[1], -it.nf[2]};
      orc_offset(p_hit, neg, ch.o);
      memcpy(ch.d, it.refr_dir, sizeof ch.d);
      ch.E = e_refr;
      ch.L = range;
      ch.g = r->g;
      ch.n_cur = it.n2;
      ch.depth = r->depth + 1;
      ch.heap = 2u * r->heap + 1u;
      ch.excl = (int32_t)j;
      trace_ray(c, &ch, ps);
    } else {
      if (e_refr > 0.5 * ecut) ps->exempt = 1;
      ps->energy[E_CUT] += e_refr;
    }
  }
}

static void do_column(scan_ctx* c, uint32_t ci) {
  const orc_params* prm = c->prm;
  uint32_t k = c->columns ? c->columns[ci] : ci;
  double* img = c->image + (size_t)ci * prm->n_bins;
  double* en = c->energy + (size_t)ci * E_NSLOTS;
  uint64_t segs = 0;
  for (uint32_t i = 0; i < prm->rays_per_beam; ++i) {
    size_t pid = (size_t)k * prm->rays_per_beam + i;
    if (c->primary_mask && !c->primary_mask[pid]) continue;
    size_t lp = (size_t)ci * prm->rays_per_beam + i;
    prim_state ps;
    ps.img = img;
    ps.energy = en;
    ps.rec = c->records ? c->records + lp * c->rec_stride : NULL;
    ps.air_rec = (c->records && (prm->flags & ORC_AIR_PATH)) ? ps.rec + c->n_heap : NULL;
    {
      /* beam axis of column k: the azimuth direction rotated by the pose */
      double phi = 2.0 * M_PI * (double)k / (double)prm->n_azimuth;
      double a0 = cos(phi), a1 = sin(phi);
      for (int a = 0; a < 3; ++a) ps.axis[a] = c->pc.R[a][0] * a0 + c->pc.R[a][1] * a1;
    }
    ps.exempt = 0;
    ps.segments = 0;
    oray r;
    primary(prm, c->pose, &c->pc, k, i, r.o, r.d, &r.g, NULL, NULL);
    r.E = (double)c->pc.E0;
    r.L = 0.0f;
    r.n_cur = 1.0f;
    r.depth = 0;
    r.heap = 1;
    r.excl = -1;
    en[E_EMITTED] += r.E;
    trace_ray(c, &r, &ps);
    if (c->exempt) c->exempt[lp] = (uint8_t)ps.exempt;
    segs += ps.segments;
  }
  c->seg_per_col[ci] = segs;
}

static void* worker(void* arg) {
  scan_ctx* c = (scan_ctx*)arg;
  for (;;) {
    uint32_t ci = __atomic_fetch_add(&c->next_col, 1u, __ATOMIC_RELAXED);
    if (ci >= c->n_columns) break;
    do_column(c, ci);
  }
  return NULL;
}

/*
 * Scan the columns listed in `columns` (all N_az columns if NULL).
 *   image    [n_columns][n_bins] float64, zeroed here
 *   records  optional [n_columns * N_s][2^B - 1] int32 in heap order
 *            (heap id 1 = primary, 2h = reflected child, 2h+1 = refracted
 *            child); entry = original triangle id, -1 for a miss, -2 for a
 *            segment that was never spawned.  With air-path returns each
 *            primary has 2 (2^B - 1) entries; the second half holds the
 *            air-path outcome of each segment's hit: -2 none attempted,
 *            0 returned, 1 blocked, 2 beyond the last bin (not tested)
 *   exempt   optional [n_columns * N_s] uint8 near-degenerate flags
 *   energy   optional [n_columns][8] float64: emitted, returned in range,
 *            returned out of range, escaped, absorbed, depth-terminated, cut,
 *            blocked air-path returns
 *   segments optional [n_columns] uint64 closest-hit queries per column
 * Returns 0, or -1 on an invalid argument.
 */
int orc_scan(const float* vertices, uint32_t nv, const uint32_t* indices, uint32_t nt,
             const uint16_t* tri_material, const orc_pose* pose, const orc_params* prm,
             const orc_material* mats, uint32_t n_mats, const uint32_t* columns,
             uint32_t n_columns, const uint8_t* primary_mask, double* image, int32_t* records,
             uint8_t* exempt, double* energy, uint64_t* segments, int n_threads) {
  if (!prm || !pose || !mats || !image || prm->max_bounces < 1 || prm->max_bounces > 8 ||
      prm->n_azimuth < 1 || prm->rays_per_beam < 1 || prm->n_bins < 1)
    return -1;
  if (!columns) n_columns = prm->n_azimuth;
  for (uint32_t ci = 0; ci < n_columns && columns; ++ci)
    if (columns[ci] >= prm->n_azimuth) return -1;
  for (uint32_t j = 0; j < nt; ++j) {
    if (tri_material[j] >= n_mats) return -1;
    for (int a = 0; a < 3; ++a)
      if (indices[3 * j + a] >= nv) return -1;
  }
  scan_ctx c;
  memset(&c, 0, sizeof c);
  c.nt = nt;
  c.v0 = malloc(sizeof(float) * 3 * (nt ? nt : 1));
  c.e1 = malloc(sizeof(float) * 3 * (nt ? nt : 1));
  c.e2 = malloc(sizeof(float) * 3 * (nt ? nt : 1));
  c.ng = malloc(sizeof(float) * 3 * (nt ? nt : 1));
  c.degenerate = malloc(nt ? nt : 1);
  c.win = malloc(sizeof(double[4]) * n_mats);
  c.seg_per_col = calloc(n_columns ? n_columns : 1, sizeof(uint64_t));
  double* en_local = energy ? NULL : calloc((size_t)(n_columns ? n_columns : 1) * E_NSLOTS, sizeof(double));
  for (uint32_t j = 0; j < nt; ++j) {
    const float* p0 = vertices + 3 * indices[3 * j + 0];
    const float* p1 = vertices + 3 * indices[3 * j + 1];
    const float* p2 = vertices + 3 * indices[3 * j + 2];
    float* v0 = c.v0 + 3 * j;
    float* e1 = c.e1 + 3 * j;
    float* e2 = c.e2 + 3 * j;
    float* n = c.ng + 3 * j;
    memcpy(v0, p0, 12);
    subf(p1, p0, e1);
    subf(p2, p0, e2);
    crossf(e1, e2, n);
    float nn = dotf(n, n);
    /* zero-area (or underflowing) triangles have no normal and are never hit */
    c.degenerate[j] = !(nn > 0.0f);
    if (!c.degenerate[j]) {
      float len = sqrtf(nn);
      n[0] = n[0] / len;
      n[1] = n[1] / len;
      n[2] = n[2] / len;
    }
  }
  c.mat = tri_material;
  c.mats = mats;
  for (uint32_t m = 0; m < n_mats; ++m) orc_window_coeffs(&mats[m], prm->beam_width_rad, c.win[m]);
  c.prm = prm;
  c.pose = pose;
  make_prim_consts(prm, pose, &c.pc);
  c.r_max = (float)prm->n_bins * prm->bin_size_m;
  c.n_heap = (1u << prm->max_bounces) - 1u;
  c.rec_stride = (prm->flags & ORC_AIR_PATH) ? 2u * c.n_heap : c.n_heap;
  c.columns = columns;
  c.n_columns = n_columns;
  c.primary_mask = primary_mask;
  c.image = image;
  c.records = records;
  c.exempt = exempt;
  c.energy = energy ? energy : en_local;
  memset(image, 0, sizeof(double) * (size_t)n_columns * prm->n_bins);
  memset(c.energy, 0, sizeof(double) * (size_t)n_columns * E_NSLOTS);
  if (records) {
    size_t nrec = (size_t)n_columns * prm->rays_per_beam * c.rec_stride;
    for (size_t q = 0; q < nrec; ++q) records[q] = -2;
  }
  if (exempt) memset(exempt, 0, (size_t)n_columns * prm->rays_per_beam);
  c.next_col = 0;
  if (n_threads <= 0) n_threads = (int)sysconf(_SC_NPROCESSORS_ONLN);
  if (n_threads < 1) n_threads = 1;
  if ((uint32_t)n_threads > n_columns) n_threads = (int)(n_columns ? n_columns : 1);
  pthread_t* th = malloc(sizeof(pthread_t) * (size_t)n_threads);
  for (int t = 1; t < n_threads; ++t) pthread_create(&th[t], NULL, worker, &c);
  worker(&c);
  for (int t = 1; t < n_threads; ++t) pthread_join(th[t], NULL);
  free(th);
  if (segments) memcpy(segments, c.seg_per_col, sizeof(uint64_t) * n_columns);
  free(c.v0);
  free(c.e1);
  free(c.e2);
  free(c.ng);
  free(c.degenerate);
  free(c.win);
  free(c.seg_per_col);
  free(en_local);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Polar-image epilogue (Sec. III-B "Polar Image", Sec. III-C "Noise"),     */
/* in float64, each step as the readings define it:                         */
/*   1. measurement noise: each azimuth column blurred along range with a   */
/*      Gaussian of std. dev. sigma bins, weights exp(-m^2 / (2 sigma^2))   */
/*      for |m| <= ceil(3 sigma), normalised to sum 1, zero beyond the ends;*/
/*   2. system noise: uniform_amp * u per pixel, u from word (bin mod 4) of */
/*      Philox with counter (k, bin div 4, 1, 0); ambient noise: perlin_amp * (0.5 + 0.5 n), n the   */
/*      2-D gradient noise of Perlin ("Improving noise", SIGGRAPH 2002) at  */
/*      (k / cell_az, bin / cell_bins), lattice gradients picked by the top */
/*      three bits of Philox (i, j, 2, 0) from the eight vectors (+-1, +-1),*/
/*      (+-1, 0), (0, +-1), fade t^3 (t (6t - 15) + 10);                    */
/*   3. L = 10 log10(E) (E_0 = 1: the image is already a fraction of each   */
/*      azimuth's emitted energy), -inf for E <= 0;                         */
/*   4. pixel = floor(max_value * (L - floor) / (0 - floor) + 0.5), clamped */
/*      to [0, max_value] (L above 0 dB is cut to max_value).               */
/* ------------------------------------------------------------------------ */
typedef struct {
  float blur_sigma_bins, uniform_amp, perlin_amp, perlin_cell_az, perlin_cell_bins, db_floor;
  uint32_t max_value, reserved0;
  uint64_t seed;
  uint32_t scan_id, reserved1;
} orc_post_params;

static double orc_u53(uint64_t x) { return (double)(x >> 11) * (1.0 / 9007199254740992.0); }

static double fade5(double t) { return t * t * t * (t * (t * 6.0 - 15.0) + 10.0); }

static double grad_dot(uint64_t key[2], int64_t i, int64_t j, double dx, double dy) {
  static const double gx[8] = {1.0, -1.0, 1.0, -1.0, 1.0, -1.0, 0.0, 0.0};
  static const double gy[8] = {1.0, 1.0, -1.0, -1.0, 0.0, 0.0, 1.0, -1.0};
  uint64_t ctr[4] = {(uint64_t)i, (uint64_t)j, 2u, 0u}, x[4];
  orc_philox4x64_10(key, ctr, x);
  unsigned g = (unsigned)(x[0] >> 61);
  return gx[g] * dx + gy[g] * dy;
}

double orc_perlin(uint64_t seed, uint32_t scan_id, double x, double y) {
  uint64_t key[2] = {seed, scan_id};
  double fx0 = floor(x), fy0 = floor(y);
  int64_t i = (int64_t)fx0, j = (int64_t)fy0;
  double fx = x - fx0, fy = y - fy0;
  double n00 = grad_dot(key, i, j, fx, fy);
  double n10 = grad_dot(key, i + 1, j, fx - 1.0, fy);
  double n01 = grad_dot(key, i, j + 1, fx, fy - 1.0);
  double n11 = grad_dot(key, i + 1, j + 1, fx - 1.0, fy - 1.0);
  double u = fade5(fx), v = fade5(fy);
  double nx0 = n00 + u * (n10 - n00);
  double nx1 = n01 + u * (n11 - n01);
  return nx0 + v * (nx1 - nx0);
}

/* db_out (float, may be NULL), u8_out (may be NULL), pre_out (may be NULL):
 * max_value * (L - floor) / (0 - floor) before rounding, for the tests. */
void orc_post(const float* image, uint32_t n_az, uint32_t n_bins, const orc_post_params* p,
              float* db_out, uint8_t* u8_out, double* pre_out) {
  double sigma = p->blur_sigma_bins;
  int R = sigma > 0.0 ? (int)ceil(3.0 * sigma) : 0;
  double* w = (double*)malloc(sizeof(double) * (size_t)(2 * R + 1));
  double wsum = 0.0;
  for (int m = -R; m <= R; ++m) {
    w[m + R] = R ? exp(-((double)m * (double)m) / (2.0 * sigma * sigma)) : 1.0;
    wsum += w[m + R];
  }
  for (int m = -R; m <= R; ++m) w[m + R] = w[m + R] / wsum;
  uint64_t key[2] = {p->seed, p->scan_id};
  double floor_db = p->db_floor;
  for (uint32_t k = 0; k < n_az; ++k) {
    for (uint32_t b = 0; b < n_bins; ++b) {
      double e = 0.0;
      for (int m = -R; m <= R; ++m) {
        long j = (long)b + m;
        if (j < 0 || j >= (long)n_bins) continue;
        e += w[m + R] * (double)image[(size_t)k * n_bins + (size_t)j];
      }
      if (p->uniform_amp > 0.0f) {
        uint64_t ctr[4] = {k, b / 4u, 1u, 0u}, x[4];
        orc_philox4x64_10(key, ctr, x);
        e += (double)p->uniform_amp * orc_u53(x[b % 4u]);
      }
      if (p->perlin_amp > 0.0f) {
        double n = orc_perlin(p->seed, p->scan_id, (double)k / (double)p->perlin_cell_az,
                              (double)b / (double)p->perlin_cell_bins);
        e += (double)p->perlin_amp * (0.5 + 0.5 * n);
      }
      double L = e > 0.0 ? 10.0 * log10(e) : -INFINITY;
      double pre = e > 0.0 ? (double)p->max_value * (L - floor_db) / (0.0 - floor_db) : -INFINITY;
      double q = floor(pre + 0.5);
      if (!(q > 0.0)) q = 0.0;
      if (q > (double)p->max_value) q = (double)p->max_value;
      size_t o = (size_t)k * n_bins + b;
      if (db_out) db_out[o] = (float)L;
      if (u8_out) u8_out[o] = (uint8_t)q;
      if (pre_out) pre_out[o] = pre;
    }
  }
  free(w);
}
