// CPU ORACLE for the selective multi-scale Gaussian rasteriser.
//
// TEST INFRASTRUCTURE ONLY.  Nothing in the product links or calls this file;
// only the tests, the smoke check and the benchmark's CPU-baseline leg may load
// it.  It shares no code, header, table or constant generator with the HIP
// library: every formula below is written out again from the paper and from
// the numerics contract both sides follow independently.
//
// What it computes (paper: "Multi-Scale 3D Gaussian Splatting for Anti-Aliased
// Rendering", CVPR 2024):
//   * EWA projection of each 3D Gaussian to a 2D Gaussian (Sec. 3.1, with the
//     merged low-pass kernel G_{V^k+V^h} of Sec. 3.2);
//   * pixel coverage S_k: the shorter of the horizontal and vertical chords
//     through the centre of the level set sigma*G = sigma_T, sigma_T = 1/255
//     (Sec. 4.1, pixel-coverage paragraph and its figure);
//   * the selection rule of Sec. 4.1 on selective rendering (the inequality on S/S^max, S/S^min and
//     S_T = 2 px) with the finest/coarsest-level exemptions, and the range
//     update with decay factors 0.95 / 1.05 (Sec. 4.1 on selective rendering, Alg. 2);
//   * tile binning into 16x16 tiles and the depth order (Sec. 3.1);
//   * front-to-back alpha compositing (Sec. 3.1/3.2), by BRUTE FORCE: every
//     pixel visits every drawable Gaussian in depth order, with no tiles.
//
// Every discrete decision (selection, tile rectangle, key, skip, clamp,
// termination) is taken in fp32 with the operation order of the numerics
// contract, because the GPU takes it in fp32.  exp and log are written out
// from Cody-Waite range reduction with Taylor / atanh-series polynomials.
// Compile with -ffp-contract=off and without fast-math.
//
// Colours use real orthonormal spherical harmonics evaluated in fp64 through
// the associated-Legendre recursion (a different route from the GPU's
// Cartesian polynomials) and are rounded to fp32.

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

extern "C" {

typedef struct {
  int64_t n;
  int sh_degree;
  int n_levels;
  const float* means;    // [3][n]
  const float* scales;   // [3][n] linear
  const float* quats;    // [4][n] w,x,y,z
  const float* opacity;  // [n]
  const float* sh;       // [(D+1)^2*3][n], plane j*3+c
  const uint8_t* level;  // [n]
  const float* s_max;    // [n]
  const float* s_min;    // [n]
} or_scene;

typedef struct {
  float R[9];
  float t[3];
  float fx, fy, cx, cy;
  int width, height;
} or_camera;

typedef struct {
  int downscale;
  int selective;
  float lowpass;
  float near_z;
  float bg[3];
} or_opts;

typedef struct {
  uint8_t* front;    // [n]
  uint8_t* sel;      // [n]  selection mask (front and Eq.C with exemptions)
  uint8_t* draw;     // [n]  selected, visible level set and invertible V'
  float* S;          // [n]  pixel coverage
  float* depth;      // [n]  view-space z
  float* V;          // [3n] V11,V12,V22 (undilated), planar
  float* u;          // [2n] projected centre
  float* conic;      // [3n] A11,A12,A22 of (V+hI)^-1
  float* lnq;        // [n]  ln(255 sigma)
  float* color;      // [3n] clamped colour
  uint8_t* cclamp;   // [3n] colour clamp flags
  int32_t* rect;     // [4n] x_lo,x_hi,y_lo,y_hi (inclusive tile indices)
  int64_t* ntiles;   // [n]
} or_proj_out;

}  // extern "C"

namespace {

// ---------------------------------------------------------------- exp / log
// Cody-Waite reduction x = n ln2 + r, |r| <= ln2/2, then exp(r) by its Taylor
// series to degree 7 in Horner form with fused multiply-adds, then 2^n.
const float kL2E = 0x1.715476p+0f;     // log2(e) rounded to fp32
const float kLn2Hi = 0x1.62e400p-1f;   // ln2 with the low 12 bits cleared
const float kLn2Lo = 0x1.7f7d1cp-20f;  // ln2 - kLn2Hi rounded to fp32

inline float exp_spec(float x) {
  float n = rintf(x * kL2E);
  float r = fmaf(n, -kLn2Hi, x);
  r = fmaf(n, -kLn2Lo, r);
  float p = 0x1.a01a02p-13f;        // 1/7!
  p = fmaf(p, r, 0x1.6c16c2p-10f);  // 1/6!
  p = fmaf(p, r, 0x1.111112p-7f);   // 1/5!
  p = fmaf(p, r, 0x1.555556p-5f);   // 1/4!
  p = fmaf(p, r, 0x1.555556p-3f);   // 1/3!
  p = fmaf(p, r, 0.5f);             // 1/2!
  p = fmaf(p, r, 1.0f);             // 1/1!
  p = fmaf(p, r, 1.0f);             // 1/0!
  return ldexpf(p, (int)n);
}

// y = m 2^e with m in [sqrt(1/2), sqrt(2)); ln m = 2 atanh(s), s = (m-1)/(m+1),
// atanh(s) = s + s^3/3 + ... + s^11/11.
inline float log_spec(float y) {
  int e = 0;
  float m = frexpf(y, &e);
  if (m < 0x1.6a09e6p-1f) {
    m = m + m;
    e = e - 1;
  }
  float f = m - 1.0f;
  float g = m + 1.0f;
  float s = f / g;
  float z = s * s;
  float p = 0x1.745d18p-4f;        // 1/11
  p = fmaf(p, z, 0x1.c71c72p-4f);  // 1/9
  p = fmaf(p, z, 0x1.24924ap-3f);  // 1/7
  p = fmaf(p, z, 0x1.99999ap-3f);  // 1/5
  p = fmaf(p, z, 0x1.555556p-2f);  // 1/3
  float t = z * p;
  float w = fmaf(s, t, s);
  float ls = w + w;
  float ef = (float)e;
  float res = fmaf(ef, kLn2Lo, ls);
  res = fmaf(ef, kLn2Hi, res);
  return res;
}

const float kAlphaMin = 0x1.010102p-8f;  // 1/255 rounded to fp32 (sigma_T)
const float kMargin = 0x1p-10f;
const float kLqPad = 0x1p-8f;

inline uint32_t fbits(float f) {
  uint32_t b;
  std::memcpy(&b, &f, 4);
  return b;
}

// ---------------------------------------------------------------- SH (fp64)
// Real orthonormal spherical harmonics without the Condon-Shortley phase:
//   Y_l^0 = K_l^0 P_l^0(cos t), Y_l^{+m} = sqrt2 K_l^m cos(m phi) P_l^m(cos t),
//   Y_l^{-m} = sqrt2 K_l^m sin(m phi) P_l^m(cos t),
//   K_l^m = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!).
// Index j = l*l + l + m.
double factorial(int k) {
  double r = 1.0;
  for (int i = 2; i <= k; ++i) r *= i;
  return r;
}

void sh_basis64(int degree, double x, double y, double z, double* out) {
  const double pi = 3.14159265358979323846;
  double ct = std::max(-1.0, std::min(1.0, z));
  double st = std::sqrt(std::max(0.0, 1.0 - ct * ct));
  double phi = std::atan2(y, x);
  // associated Legendre P_l^m(ct) without the (-1)^m phase
  double P[4][4] = {{0}};
  for (int m = 0; m <= degree; ++m) {
    double pmm = 1.0;
    for (int i = 1; i <= m; ++i) pmm *= (2.0 * i - 1.0) * st;
    P[m][m] = pmm;
    if (m + 1 <= degree) P[m + 1][m] = ct * (2.0 * m + 1.0) * pmm;
    for (int l = m + 2; l <= degree; ++l)
      P[l][m] = ((2.0 * l - 1.0) * ct * P[l - 1][m] - (l + m - 1.0) * P[l - 2][m]) / (l - m);
  }
  for (int l = 0; l <= degree; ++l) {
    for (int m = -l; m <= l; ++m) {
      int am = m < 0 ? -m : m;
      double K = std::sqrt((2.0 * l + 1.0) / (4.0 * pi) * factorial(l - am) / factorial(l + am));
      double v;
      if (m == 0)
        v = K * P[l][0];
      else if (m > 0)
        v = std::sqrt(2.0) * K * std::cos(m * phi) * P[l][m];
      else
        v = std::sqrt(2.0) * K * std::sin(am * phi) * P[l][am];
      out[l * l + l + m] = v;
    }
  }
}

// ---------------------------------------------------------------- camera
struct Cam {
  float R[9], t[3];
  float fx, fy, cx, cy;
  int W, H, Tx, Ty;
  double C[3];  // camera centre -R^T t (fp64)
};

bool make_cam(const or_camera* c, const or_opts* o, Cam* k) {
  if (o->downscale < 1) return false;
  // a camera with a non-finite entry is rejected: with a NaN centre every skip
  // test of the compositing is false, so nothing bounds the drawn pixels
  for (int i = 0; i < 9; ++i)
    if (!std::isfinite(c->R[i])) return false;
  for (int i = 0; i < 3; ++i)
    if (!std::isfinite(c->t[i])) return false;
  if (!std::isfinite(c->fx) || !std::isfinite(c->fy) || !std::isfinite(c->cx) ||
      !std::isfinite(c->cy))
    return false;
  std::memcpy(k->R, c->R, sizeof k->R);
  std::memcpy(k->t, c->t, sizeof k->t);
  float d = (float)o->downscale;
  k->fx = c->fx / d;
  k->fy = c->fy / d;
  k->cx = c->cx / d;
  k->cy = c->cy / d;
  k->W = c->width / o->downscale;
  k->H = c->height / o->downscale;
  if (k->W <= 0 || k->H <= 0) return false;
  k->Tx = (k->W + 15) / 16;
  k->Ty = (k->H + 15) / 16;
  for (int i = 0; i < 3; ++i)
    k->C[i] = -((double)c->R[0 * 3 + i] * c->t[0] + (double)c->R[1 * 3 + i] * c->t[1] +
                (double)c->R[2 * 3 + i] * c->t[2]);
  return true;
}

// ---------------------------------------------------------------- projection
struct Proj {
  bool front = false, vis = false, sel = false, draw = false;
  float p[3] = {0, 0, 0};
  float V11 = 0, V12 = 0, V22 = 0;
  float S = 0, lnq = 0, lq = 0, sigma = 0;
  float ux = 0, uy = 0;
  float A11 = 0, A12 = 0, A22 = 0;
  int rect[4] = {0, -1, 0, -1};
  int64_t ntiles = 0;
  float col[3] = {0, 0, 0};
  bool cclamp[3] = {false, false, false};
};

// fmin/fmax semantics: a NaN operand yields the other operand.
float clampf_to(float v, float lo, float hi) { return fminf(fmaxf(v, lo), hi); }

void project_one(const or_scene* s, const Cam& cam, const or_opts* o, int64_t k, Proj* P) {
  const int64_t n = s->n;
  // rotation from the normalised quaternion
  float qw = s->quats[0 * n + k], qx = s->quats[1 * n + k];
  float qy = s->quats[2 * n + k], qz = s->quats[3 * n + k];
  float nrm2 = ((qw * qw + qx * qx) + qy * qy) + qz * qz;
  float r = sqrtf(nrm2);
  float w = qw / r, x = qx / r, y = qy / r, z = qz / r;
  float Q[9];
  Q[0] = 1.0f - 2.0f * (y * y + z * z);
  Q[1] = 2.0f * (x * y - w * z);
  Q[2] = 2.0f * (x * z + w * y);
  Q[3] = 2.0f * (x * y + w * z);
  Q[4] = 1.0f - 2.0f * (x * x + z * z);
  Q[5] = 2.0f * (y * z - w * x);
  Q[6] = 2.0f * (x * z - w * y);
  Q[7] = 2.0f * (y * z + w * x);
  Q[8] = 1.0f - 2.0f * (x * x + y * y);
  float sc[3] = {s->scales[0 * n + k], s->scales[1 * n + k], s->scales[2 * n + k]};
  float M[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) M[i * 3 + j] = Q[i * 3 + j] * sc[j];
  // Sigma = M M^T (symmetric; Sg[i][j] for i <= j)
  float Sg[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = i; j < 3; ++j) {
      Sg[i][j] = (M[i * 3 + 0] * M[j * 3 + 0] + M[i * 3 + 1] * M[j * 3 + 1]) + M[i * 3 + 2] * M[j * 3 + 2];
      Sg[j][i] = Sg[i][j];
    }
  // view transform
  float mu[3] = {s->means[0 * n + k], s->means[1 * n + k], s->means[2 * n + k]};
  for (int i = 0; i < 3; ++i)
    P->p[i] = ((cam.R[i * 3 + 0] * mu[0] + cam.R[i * 3 + 1] * mu[1]) + cam.R[i * 3 + 2] * mu[2]) + cam.t[i];
  float px = P->p[0], py = P->p[1], pz = P->p[2];
  P->front = pz > o->near_z;
  if (!P->front) return;
  // Jacobian of the perspective map at p
  float z2 = pz * pz;
  float J00 = cam.fx / pz;
  float J02 = -((cam.fx * px) / z2);
  float J11 = cam.fy / pz;
  float J12 = -((cam.fy * py) / z2);
  float Tm[2][3];
  for (int j = 0; j < 3; ++j) {
    Tm[0][j] = J00 * cam.R[0 * 3 + j] + J02 * cam.R[2 * 3 + j];
    Tm[1][j] = J11 * cam.R[1 * 3 + j] + J12 * cam.R[2 * 3 + j];
  }
  float U[2][3];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 3; ++j)
      U[i][j] = (Tm[i][0] * Sg[0][j] + Tm[i][1] * Sg[1][j]) + Tm[i][2] * Sg[2][j];
  P->V11 = (U[0][0] * Tm[0][0] + U[0][1] * Tm[0][1]) + U[0][2] * Tm[0][2];
  P->V12 = (U[0][0] * Tm[1][0] + U[0][1] * Tm[1][1]) + U[0][2] * Tm[1][2];
  P->V22 = (U[1][0] * Tm[1][0] + U[1][1] * Tm[1][1]) + U[1][2] * Tm[1][2];
  P->ux = (cam.fx * px) / pz + cam.cx;
  P->uy = (cam.fy * py) / pz + cam.cy;
  // density level set sigma G = sigma_T exists iff 255 sigma > 1
  float sig = s->opacity[k];
  P->sigma = sig;
  float y255 = 255.0f * sig;
  P->vis = y255 > 1.0f;
  P->lnq = P->vis ? log_spec(y255) : 0.0f;
  // pixel coverage: S^2 = 8 lnq det(V) / max(V11, V22)
  float det = P->V11 * P->V22 - P->V12 * P->V12;
  float mx = fmaxf(P->V11, P->V22);
  if (P->vis && det > 0.0f && mx > 0.0f) {
    float t8 = 8.0f * P->lnq;
    t8 = t8 * det;
    t8 = t8 / mx;
    P->S = sqrtf(t8);
  } else {
    P->S = 0.0f;
  }
  // selection with the finest / coarsest exemptions
  bool sel = true;
  if (o->selective) {
    int l = s->level[k];
    bool g1 = (l == 0) || (P->S <= 1.5f * s->s_max[k]);
    bool g2 = (l == s->n_levels - 1) || (P->S >= 0.5f * s->s_min[k]) || (P->S >= 2.0f);
    sel = g1 && g2;
  }
  P->sel = sel;
  if (!sel || !P->vis) return;
  // dilated covariance and its inverse (the conic)
  float W11 = P->V11 + o->lowpass;
  float W22 = P->V22 + o->lowpass;
  float W12 = P->V12;
  float det2 = W11 * W22 - W12 * W12;
  if (!(det2 > 0.0f)) return;
  P->A11 = W22 / det2;
  P->A12 = -(W12 / det2);
  P->A22 = W11 / det2;
  P->draw = true;
  // conservative extent of the level set of the drawn Gaussian
  P->lq = P->lnq + kLqPad;
  float ex = sqrtf((2.0f * P->lq) * W11) * (1.0f + kMargin) + kMargin;
  float ey = sqrtf((2.0f * P->lq) * W22) * (1.0f + kMargin) + kMargin;
  float xl = ceilf(((P->ux - ex) - 15.5f) * 0.0625f);
  float xh = floorf(((P->ux + ex) - 0.5f) * 0.0625f);
  float yl = ceilf(((P->uy - ey) - 15.5f) * 0.0625f);
  float yh = floorf(((P->uy + ey) - 0.5f) * 0.0625f);
  int ixl = std::max(0, (int)clampf_to(xl, -1.0f, (float)cam.Tx));
  int ixh = std::min(cam.Tx - 1, (int)clampf_to(xh, -1.0f, (float)cam.Tx));
  int iyl = std::max(0, (int)clampf_to(yl, -1.0f, (float)cam.Ty));
  int iyh = std::min(cam.Ty - 1, (int)clampf_to(yh, -1.0f, (float)cam.Ty));
  P->rect[0] = ixl;
  P->rect[1] = ixh;
  P->rect[2] = iyl;
  P->rect[3] = iyh;
  int64_t nx = std::max(0, ixh - ixl + 1), ny = std::max(0, iyh - iyl + 1);
  P->ntiles = nx * ny;
  // colour: SH in fp64 towards the view direction, offset 0.5, clamped at 0
  double dir[3];
  double nn = 0.0;
  for (int i = 0; i < 3; ++i) {
    dir[i] = (double)mu[i] - cam.C[i];
    nn += dir[i] * dir[i];
  }
  nn = std::sqrt(nn);
  for (int i = 0; i < 3; ++i) dir[i] /= nn;
  int D = s->sh_degree;
  int K = (D + 1) * (D + 1);
  double Y[16];
  sh_basis64(D, dir[0], dir[1], dir[2], Y);
  for (int c = 0; c < 3; ++c) {
    double v = 0.5;
    for (int j = 0; j < K; ++j) v += Y[j] * (double)s->sh[(int64_t)(j * 3 + c) * n + k];
    P->cclamp[c] = v < 0.0;
    P->col[c] = (float)(v < 0.0 ? 0.0 : v);
  }
}

void project_all(const or_scene* s, const Cam& cam, const or_opts* o, std::vector<Proj>& P) {
  P.assign((size_t)s->n, Proj());
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < s->n; ++k) project_one(s, cam, o, k, &P[k]);
}

// drawable Gaussians ordered by (depth bits, index)
std::vector<int64_t> depth_order(const std::vector<Proj>& P) {
  std::vector<int64_t> L;
  for (int64_t k = 0; k < (int64_t)P.size(); ++k)
    if (P[k].draw) L.push_back(k);
  std::stable_sort(L.begin(), L.end(), [&](int64_t a, int64_t b) {
    return fbits(P[a].p[2]) < fbits(P[b].p[2]);
  });
  return L;
}

struct PixOut {
  float rgb[3];
  float T;
  uint32_t n;
};

// Front-to-back compositing of one pixel over every drawable Gaussian in depth
// order.  When `trace` is non-null the accumulated contributors and their
// alpha-clamp flag are appended to it.
PixOut composite(const std::vector<Proj>& P, const std::vector<int64_t>& L, int i, int j,
                 const float* bg, std::vector<std::pair<int64_t, uint8_t>>* trace) {
  float pcx = (float)i + 0.5f;
  float pcy = (float)j + 0.5f;
  float T = 1.0f;
  float C[3] = {0.0f, 0.0f, 0.0f};
  uint32_t cnt = 0;
  for (int64_t k : L) {
    const Proj& g = P[k];
    float dx = pcx - g.ux;
    float dy = pcy - g.uy;
    float qx = dx * dx, qy = dy * dy, qxy = dx * dy;
    float a = g.A11 * qx;
    float b = g.A22 * qy;
    float c = a + b;
    float e = -0.5f * c;
    float f = g.A12 * qxy;
    float power = e - f;
    if (power > 0.0f) continue;
    if (power < -g.lq) continue;  // alpha is certainly below 1/255 here
    float ar = g.sigma * exp_spec(power);
    if (ar < kAlphaMin) continue;
    float al = fminf(0.99f, ar);
    float Tn = T * (1.0f - al);
    if (Tn < 1e-4f) break;
    float wgt = al * T;
    for (int ch = 0; ch < 3; ++ch) C[ch] = C[ch] + g.col[ch] * wgt;
    T = Tn;
    ++cnt;
    if (trace) trace->push_back({k, (uint8_t)(ar > 0.99f ? 1 : 0)});
  }
  PixOut o;
  for (int ch = 0; ch < 3; ++ch) o.rgb[ch] = C[ch] + T * bg[ch];
  o.T = T;
  o.n = cnt;
  return o;
}

void set_threads(int nthreads) {
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#else
  (void)nthreads;
#endif
}

}  // namespace

extern "C" {

int or_version(void) { return 1; }

// The tile-index conversion of the rectangle rule: clamp to [-1, T] with
// fmin/fmax semantics (a NaN operand yields the bound), then truncate.
int or_clamp_tile(float v, int T) { return (int)clampf_to(v, -1.0f, (float)T); }

int or_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void or_exp_spec(const float* x, float* y, int64_t n) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) y[i] = exp_spec(x[i]);
}

void or_log_spec(const float* x, float* y, int64_t n) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) y[i] = log_spec(x[i]);
}

// fp64 real SH basis at unit directions dirs[3][m] -> out[(D+1)^2][m]
void or_sh_basis(int degree, const double* dirs, int64_t m, double* out) {
  int K = (degree + 1) * (degree + 1);
  for (int64_t i = 0; i < m; ++i) {
    double Y[16];
    sh_basis64(degree, dirs[i], dirs[m + i], dirs[2 * m + i], Y);
    for (int j = 0; j < K; ++j) out[j * m + i] = Y[j];
  }
}

// Per-Gaussian projection, coverage, selection, conic, rectangle and colour.
int or_project(const or_scene* s, const or_camera* c, const or_opts* o, or_proj_out* out,
               int nthreads) {
  Cam cam;
  if (!make_cam(c, o, &cam)) return -1;
  set_threads(nthreads);
  std::vector<Proj> P;
  project_all(s, cam, o, P);
  const int64_t n = s->n;
  for (int64_t k = 0; k < n; ++k) {
    const Proj& g = P[k];
    if (out->front) out->front[k] = g.front;
    if (out->sel) out->sel[k] = g.front && g.sel;
    if (out->draw) out->draw[k] = g.draw;
    if (out->S) out->S[k] = g.S;
    if (out->depth) out->depth[k] = g.p[2];
    if (out->V) {
      out->V[k] = g.V11;
      out->V[n + k] = g.V12;
      out->V[2 * n + k] = g.V22;
    }
    if (out->u) {
      out->u[k] = g.ux;
      out->u[n + k] = g.uy;
    }
    if (out->conic) {
      out->conic[k] = g.A11;
      out->conic[n + k] = g.A12;
      out->conic[2 * n + k] = g.A22;
    }
    if (out->lnq) out->lnq[k] = g.lnq;
    for (int ch = 0; ch < 3; ++ch) {
      if (out->color) out->color[ch * n + k] = g.col[ch];
      if (out->cclamp) out->cclamp[ch * n + k] = g.cclamp[ch];
    }
    if (out->rect)
      for (int q = 0; q < 4; ++q) out->rect[q * n + k] = g.rect[q];
    if (out->ntiles) out->ntiles[k] = g.draw ? g.ntiles : 0;
  }
  return 0;
}

// Sorted (tile, depth) keys.  Emission: Gaussians in index order, tiles of each
// rectangle row-major; key = tile_id * 2^32 + bits(depth); value = Gaussian
// index; stable sort on the key.  Returns the instance count; fills the
// outputs only when cap >= count.
int64_t or_keys(const or_scene* s, const or_camera* c, const or_opts* o, uint64_t* keys,
                uint32_t* vals, int64_t cap, int nthreads) {
  Cam cam;
  if (!make_cam(c, o, &cam)) return -1;
  set_threads(nthreads);
  std::vector<Proj> P;
  project_all(s, cam, o, P);
  int64_t total = 0;
  for (const Proj& g : P)
    if (g.draw) total += g.ntiles;
  if (cap < total || keys == nullptr || vals == nullptr) return total;
  std::vector<std::pair<uint64_t, uint32_t>> E;
  E.reserve((size_t)total);
  for (int64_t k = 0; k < s->n; ++k) {
    const Proj& g = P[k];
    if (!g.draw || g.ntiles == 0) continue;
    for (int ty = g.rect[2]; ty <= g.rect[3]; ++ty)
      for (int tx = g.rect[0]; tx <= g.rect[1]; ++tx) {
        uint64_t tile = (uint64_t)ty * (uint64_t)cam.Tx + (uint64_t)tx;
        E.push_back({(tile << 32) | (uint64_t)fbits(g.p[2]), (uint32_t)k});
      }
  }
  std::stable_sort(E.begin(), E.end(),
                   [](const std::pair<uint64_t, uint32_t>& a, const std::pair<uint64_t, uint32_t>& b) {
                     return a.first < b.first;
                   });
  for (int64_t i = 0; i < total; ++i) {
    keys[i] = E[i].first;
    vals[i] = E[i].second;
  }
  return total;
}

// Brute-force image: every pixel composites every drawable Gaussian in depth
// order.  rgb [H_d][W_d][3], T_final [H_d][W_d], n_contrib [H_d][W_d].
int or_render(const or_scene* s, const or_camera* c, const or_opts* o, float* rgb, float* Tf,
              uint32_t* ncontrib, int64_t* blends, int nthreads) {
  Cam cam;
  if (!make_cam(c, o, &cam)) return -1;
  set_threads(nthreads);
  std::vector<Proj> P;
  project_all(s, cam, o, P);
  std::vector<int64_t> L = depth_order(P);
  const int W = cam.W, H = cam.H;
  int64_t tot = 0;
#pragma omp parallel for schedule(dynamic, 4) reduction(+ : tot)
  for (int64_t pix = 0; pix < (int64_t)W * H; ++pix) {
    int i = (int)(pix % W), j = (int)(pix / W);
    PixOut r = composite(P, L, i, j, o->bg, nullptr);
    for (int ch = 0; ch < 3; ++ch) rgb[pix * 3 + ch] = r.rgb[ch];
    if (Tf) Tf[pix] = r.T;
    if (ncontrib) ncontrib[pix] = r.n;
    tot += r.n;
  }
  if (blends) *blends = tot;
  return 0;
}

// Brute-force compositing of a list of pixels given as (x, y) pairs.
int or_render_pixels(const or_scene* s, const or_camera* c, const or_opts* o, int64_t npx,
                     const int32_t* pix, float* rgb, float* Tf, uint32_t* ncontrib, int nthreads) {
  Cam cam;
  if (!make_cam(c, o, &cam)) return -1;
  set_threads(nthreads);
  std::vector<Proj> P;
  project_all(s, cam, o, P);
  std::vector<int64_t> L = depth_order(P);
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t q = 0; q < npx; ++q) {
    PixOut r = composite(P, L, pix[2 * q], pix[2 * q + 1], o->bg, nullptr);
    for (int ch = 0; ch < 3; ++ch) rgb[q * 3 + ch] = r.rgb[ch];
    if (Tf) Tf[q] = r.T;
    if (ncontrib) ncontrib[q] = r.n;
  }
  return 0;
}

// Contributor trace of a list of pixels: CSR offsets [npx+1], Gaussian indices
// and alpha-clamp flags in compositing order.  Returns the total length; fills
// the lists only when cap >= total.
int64_t or_trace(const or_scene* s, const or_camera* c, const or_opts* o, int64_t npx,
                 const int32_t* pix, int64_t cap, int64_t* off, int64_t* ks, uint8_t* flags,
                 int nthreads) {
  Cam cam;
  if (!make_cam(c, o, &cam)) return -1;
  set_threads(nthreads);
  std::vector<Proj> P;
  project_all(s, cam, o, P);
  std::vector<int64_t> L = depth_order(P);
  std::vector<std::vector<std::pair<int64_t, uint8_t>>> tr((size_t)npx);
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t q = 0; q < npx; ++q) composite(P, L, pix[2 * q], pix[2 * q + 1], o->bg, &tr[q]);
  int64_t total = 0;
  for (auto& v : tr) total += (int64_t)v.size();
  if (cap < total || off == nullptr) return total;
  int64_t pos = 0;
  for (int64_t q = 0; q < npx; ++q) {
    off[q] = pos;
    for (auto& e : tr[q]) {
      ks[pos] = e.first;
      flags[pos] = e.second;
      ++pos;
    }
  }
  off[npx] = pos;
  return total;
}

// Range update at this camera (Sec. 4.1 on selective rendering): for Gaussians in front of the camera
// whose level l has creation downscale 4^l equal to the render downscale,
// S^max <- max(0.95 S^max, S) and S^min <- min(1.05 S^min, S).  s_max/s_min
// are updated in place in the caller's arrays (the scene's own pointers are
// only read).
int or_update_range(const or_scene* s, const or_camera* c, const or_opts* o, float* s_max,
                    float* s_min, int nthreads) {
  Cam cam;
  if (!make_cam(c, o, &cam)) return -1;
  set_threads(nthreads);
  std::vector<Proj> P;
  project_all(s, cam, o, P);
  int lr = -1;
  for (int l = 0, sc = 1; l < s->n_levels; ++l, sc *= 4)
    if (sc == o->downscale) lr = l;
  if (lr < 0) return 0;
  for (int64_t k = 0; k < s->n; ++k) {
    if (!P[k].front || s->level[k] != lr) continue;
    s_max[k] = fmaxf(0.95f * s_max[k], P[k].S);
    s_min[k] = fminf(1.05f * s_min[k], P[k].S);
  }
  return 0;
}

}  // extern "C"
