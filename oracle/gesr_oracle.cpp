// FP64 CPU oracle for the generalized-exponential-splat (GES) rasterizer.
//
// TEST INFRASTRUCTURE ONLY.  Nothing in the product path links, loads or calls
// this file; only the tests, the smoke check and the CPU-baseline leg of the
// benchmark do.  It shares no code, header or constant table with the HIP
// library: it is written from the paper's equations and the readings listed
// next to each function.
//
// Paper passages followed (DyGASR, arXiv 2411.09156):
//   * GEF / GES falloff: Sec. 3.2, Eq. (1)-(3).  In screen space a splat at
//     squared Mahalanobis distance q contributes exp(-kappa * q^(beta/2));
//     kappa = 1/2 reproduces Eq. (3), beta = 2 is the Gaussian of Eq. (2).
//   * Covariance Sigma = R S S^T R^T: Eq. (4).
//   * Screen covariance Sigma' = J W Sigma W^T J^T: Sec. 3.2 (after Eq. 4).
//   * Shape-modulated scale gamma_hat = phi(eps) gamma, Eq. (6)-(7); phi is
//     read as 2 / (1 + exp(-rho (beta - 2))) so that phi(2) = 1.
//   * Volume rendering, Eq. (5), evaluated as discrete front-to-back alpha
//     blending (the "alpha-blending coefficients" of Sec. 3.3).
//   * Depth maps of the extended rasterizer (Sec. 3.3, mesh extraction): the
//     splat depth and a unit opacity composited like a colour over a zero
//     background (the paper names the depth map, not its formula; this is the
//     reading used).
//
// Everything is double precision.  Inputs arrive as float32 and are promoted
// exactly.  The projection is written once as a template over the scalar
// type: with `double` it is the forward; with a forward-mode dual number it
// yields the exact Jacobian of every projected quantity, which is how the
// projection adjoint is obtained (no hand-derived chain rule).  The render
// adjoint uses explicit per-pixel fragment lists (no transmittance division).

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <numeric>
#include <vector>

#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

// ---------------------------------------------------------------- settings
struct Settings {
    double kappa, rho, alpha_min, alpha_max, t_min, blur, znear, clip_fac;
    double bg[3];
    int tile_w, tile_h, sh_degree;
    // Parity model: multiplier of the derived float32 bands of the skip and
    // termination decisions (frag_band); 1 unless a test widens them.
    double band_scale;
};

Settings read_settings(const double* s) {
    Settings o;
    o.kappa = s[0]; o.rho = s[1]; o.alpha_min = s[2]; o.alpha_max = s[3]; o.t_min = s[4];
    o.blur = s[5]; o.znear = s[6]; o.clip_fac = s[7];
    o.bg[0] = s[8]; o.bg[1] = s[9]; o.bg[2] = s[10];
    o.tile_w = (int)s[11]; o.tile_h = (int)s[12]; o.sh_degree = (int)s[13];
    o.band_scale = s[14] > 0.0 ? s[14] : 1.0;
    return o;
}

struct View {
    int W, H;
    double fx, fy, cx, cy;
    double R[9];   // world -> camera rotation, row-major
    double t[3];
    double campos[3];
    int tiles_x, tiles_y;
    long tile_base;  // first global tile id of this view
    long pix_base;   // first pixel of this view in the concatenated outputs
};

std::vector<View> read_views(const double* v, int V, int tile_w, int tile_h) {
    std::vector<View> out(V);
    long tb = 0, pb = 0;
    for (int k = 0; k < V; ++k) {
        const double* a = v + 24 * k;
        View& w = out[k];
        w.W = (int)a[0]; w.H = (int)a[1];
        w.fx = a[2]; w.fy = a[3]; w.cx = a[4]; w.cy = a[5];
        for (int j = 0; j < 9; ++j) w.R[j] = a[6 + j];
        for (int j = 0; j < 3; ++j) w.t[j] = a[15 + j];
        for (int j = 0; j < 3; ++j) w.campos[j] = a[18 + j];
        w.tiles_x = (w.W + tile_w - 1) / tile_w;
        w.tiles_y = (w.H + tile_h - 1) / tile_h;
        w.tile_base = tb;
        w.pix_base = pb;
        tb += (long)w.tiles_x * w.tiles_y;
        pb += (long)w.W * w.H;
    }
    return out;
}

// ------------------------------------------------------------- dual numbers
// Forward-mode dual number with D tangent directions.
template <int D>
struct Dual {
    double v;
    double d[D];
    Dual() : v(0) { std::fill(d, d + D, 0.0); }
    Dual(double x) : v(x) { std::fill(d, d + D, 0.0); }  // NOLINT: constants promote
    static Dual var(double x, int k) { Dual r(x); r.d[k] = 1.0; return r; }
};

template <int D> Dual<D> operator+(const Dual<D>& a, const Dual<D>& b) {
    Dual<D> r(a.v + b.v); for (int k = 0; k < D; ++k) r.d[k] = a.d[k] + b.d[k]; return r;
}
template <int D> Dual<D> operator-(const Dual<D>& a, const Dual<D>& b) {
    Dual<D> r(a.v - b.v); for (int k = 0; k < D; ++k) r.d[k] = a.d[k] - b.d[k]; return r;
}
template <int D> Dual<D> operator-(const Dual<D>& a) {
    Dual<D> r(-a.v); for (int k = 0; k < D; ++k) r.d[k] = -a.d[k]; return r;
}
template <int D> Dual<D> operator*(const Dual<D>& a, const Dual<D>& b) {
    Dual<D> r(a.v * b.v); for (int k = 0; k < D; ++k) r.d[k] = a.d[k] * b.v + a.v * b.d[k]; return r;
}
template <int D> Dual<D> operator/(const Dual<D>& a, const Dual<D>& b) {
    Dual<D> r(a.v / b.v);
    for (int k = 0; k < D; ++k) r.d[k] = (a.d[k] * b.v - a.v * b.d[k]) / (b.v * b.v);
    return r;
}
template <int D> Dual<D> operator+(const Dual<D>& a, double b) { return a + Dual<D>(b); }
template <int D> Dual<D> operator+(double a, const Dual<D>& b) { return Dual<D>(a) + b; }
template <int D> Dual<D> operator-(const Dual<D>& a, double b) { return a - Dual<D>(b); }
template <int D> Dual<D> operator-(double a, const Dual<D>& b) { return Dual<D>(a) - b; }
template <int D> Dual<D> operator*(const Dual<D>& a, double b) { return a * Dual<D>(b); }
template <int D> Dual<D> operator*(double a, const Dual<D>& b) { return Dual<D>(a) * b; }
template <int D> Dual<D> operator/(const Dual<D>& a, double b) { return a / Dual<D>(b); }
template <int D> Dual<D> operator/(double a, const Dual<D>& b) { return Dual<D>(a) / b; }

template <int D> Dual<D> sqrt(const Dual<D>& a) {
    double s = std::sqrt(a.v);
    Dual<D> r(s); for (int k = 0; k < D; ++k) r.d[k] = a.d[k] / (2.0 * s); return r;
}
template <int D> Dual<D> exp(const Dual<D>& a) {
    double e = std::exp(a.v);
    Dual<D> r(e); for (int k = 0; k < D; ++k) r.d[k] = a.d[k] * e; return r;
}

inline double val(double x) { return x; }
template <int D> double val(const Dual<D>& x) { return x.v; }
using std::exp;
using std::sqrt;

// ------------------------------------------------- real spherical harmonics
// Real SH with the Condon-Shortley phase kept, index l*l + l + m, m = -l..l:
//   m > 0 : sqrt(2) K_l^m P_l^m(cos th) cos(m ph)
//   m < 0 : sqrt(2) K_l^|m| P_l^|m|(cos th) sin(|m| ph)
//   m = 0 : K_l^0 P_l(cos th)
// with K_l^m = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!) and P_l^m carrying (-1)^m.
// For a unit direction (x, y, z) = (sin th cos ph, sin th sin ph, cos th):
//   P_l^m(z) = (-1)^m (1 - z^2)^(m/2) d^m/dz^m P_l(z),
//   (1 - z^2)^(m/2) cos(m ph) = Re (x + i y)^m,  ... sin(m ph) = Im (x + i y)^m,
// so every basis function is a polynomial in (x, y, z) and the derivative with
// respect to the direction follows from the dual arithmetic.
double factorial(int n) { double f = 1; for (int i = 2; i <= n; ++i) f *= i; return f; }
double binom(int n, int k) { return factorial(n) / (factorial(k) * factorial(n - k)); }

// m-th derivative of the Legendre polynomial P_l at z, from
// P_l(z) = 2^-l sum_k (-1)^k C(l,k) C(2l-2k,l) z^(l-2k).
template <class S> S legendre_deriv(int l, int m, const S& z) {
    S acc(0.0);
    for (int k = 0; 2 * k <= l; ++k) {
        int p = l - 2 * k;
        if (p < m) continue;
        double c = std::ldexp(1.0, -l) * ((k & 1) ? -1.0 : 1.0) * binom(l, k) * binom(2 * l - 2 * k, l) *
                   factorial(p) / factorial(p - m);
        S term(c);
        for (int e = 0; e < p - m; ++e) term = term * z;
        acc = acc + term;
    }
    return acc;
}

template <class S> void sh_basis(int degree, const S& x, const S& y, const S& z, S* out) {
    const double pi = 3.14159265358979323846;
    for (int l = 0; l <= degree; ++l) {
        for (int m = -l; m <= l; ++m) {
            int am = m < 0 ? -m : m;
            double K = std::sqrt((2.0 * l + 1.0) / (4.0 * pi) * factorial(l - am) / factorial(l + am));
            S pd = legendre_deriv<S>(l, am, z);
            // (x + i y)^am
            S re(1.0), im(0.0);
            for (int e = 0; e < am; ++e) {
                S nr = re * x - im * y;
                S ni = re * y + im * x;
                re = nr; im = ni;
            }
            double phase = (am & 1) ? -1.0 : 1.0;
            S Y;
            if (m == 0) Y = K * pd;
            else if (m > 0) Y = (std::sqrt(2.0) * K * phase) * pd * re;
            else Y = (std::sqrt(2.0) * K * phase) * pd * im;
            out[l * l + l + m] = Y;
        }
    }
}

// ------------------------------------------------------------- projection
enum Cull : uint8_t { KEEP = 0, CULL_NEAR = 1, CULL_DET = 2, CULL_OPACITY = 3, CULL_EMPTY = 4, CULL_NONFINITE = 5 };

template <class S>
struct Proj {
    S u, v, A, B, C, o, beta, rgb[3];
    S z;  // camera-space depth of the centre (the extended rasterizer's depth channel)
    double depth = 0, qmax = 0, sig[3] = {0, 0, 0}, edges[4] = {0, 0, 0, 0};
    int pix[4] = {-1, -1, -2, -2}, tiles[4] = {-1, -1, -2, -2};
    uint32_t touched = 0;
    uint8_t cull = KEEP, clamp = 0;
};

// Projects one splat into one view.  `mean`, `scale`, `quat`, `opac`, `beta`
// are scalars of type S (double, or duals carrying the Jacobian); `sh` points
// at K*3 coefficients (colour is linear in them).
template <class S>
Proj<S> project_one(const S mean[3], const S scale[3], const S quat[4], const S& opac, const S& beta,
                    const double* sh, const View& vw, const Settings& st) {
    Proj<S> r;
    // camera-space position: p = W mu + t  (W is the view rotation)
    S p[3];
    for (int a = 0; a < 3; ++a)
        p[a] = vw.R[3 * a + 0] * mean[0] + vw.R[3 * a + 1] * mean[1] + vw.R[3 * a + 2] * mean[2] + vw.t[a];
    r.depth = val(p[2]);
    r.z = p[2];
    if (!(val(p[2]) > st.znear)) { r.cull = std::isfinite(val(p[2])) ? CULL_NEAR : CULL_NONFINITE; return r; }

    // rotation of the normalised quaternion (w, x, y, z), Eq. (4)
    S qn = sqrt(quat[0] * quat[0] + quat[1] * quat[1] + quat[2] * quat[2] + quat[3] * quat[3]);
    S w = quat[0] / qn, x = quat[1] / qn, y = quat[2] / qn, z = quat[3] / qn;
    S Rq[9] = {
        1.0 - 2.0 * (y * y + z * z), 2.0 * (x * y - w * z),       2.0 * (x * z + w * y),
        2.0 * (x * y + w * z),       1.0 - 2.0 * (x * x + z * z), 2.0 * (y * z - w * x),
        2.0 * (x * z - w * y),       2.0 * (y * z + w * x),       1.0 - 2.0 * (x * x + y * y)};

    // shape-modulated scale, Eq. (6)-(7): gamma_hat = phi(beta) gamma
    S phi = 2.0 / (1.0 + exp(-st.rho * (beta - 2.0)));
    S M[9];  // M = R diag(phi s)
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) M[3 * a + b] = Rq[3 * a + b] * (phi * scale[b]);
    S Sig[9];  // Sigma = M M^T
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) Sig[3 * a + b] = M[3 * a] * M[3 * b] + M[3 * a + 1] * M[3 * b + 1] + M[3 * a + 2] * M[3 * b + 2];

    // perspective Jacobian J at the (frustum-clamped) centre
    double limx = st.clip_fac * vw.W / (2.0 * vw.fx), limy = st.clip_fac * vw.H / (2.0 * vw.fy);
    S txz = p[0] / p[2], tyz = p[1] / p[2];
    S xt = (val(txz) > limx) ? S(limx) * p[2] : (val(txz) < -limx) ? S(-limx) * p[2] : p[0];
    S yt = (val(tyz) > limy) ? S(limy) * p[2] : (val(tyz) < -limy) ? S(-limy) * p[2] : p[1];
    S J[6] = {vw.fx / p[2], S(0.0), -vw.fx * xt / (p[2] * p[2]),
              S(0.0), vw.fy / p[2], -vw.fy * yt / (p[2] * p[2])};
    S T[6];  // T = J W
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 3; ++b)
            T[3 * a + b] = J[3 * a] * vw.R[b] + J[3 * a + 1] * vw.R[3 + b] + J[3 * a + 2] * vw.R[6 + b];
    // Sigma' = T Sigma T^T + blur I
    S TS[6];
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 3; ++b)
            TS[3 * a + b] = T[3 * a] * Sig[b] + T[3 * a + 1] * Sig[3 + b] + T[3 * a + 2] * Sig[6 + b];
    S sa = TS[0] * T[0] + TS[1] * T[1] + TS[2] * T[2] + st.blur;
    S sb = TS[0] * T[3] + TS[1] * T[4] + TS[2] * T[5];
    S sc = TS[3] * T[3] + TS[4] * T[4] + TS[5] * T[5] + st.blur;
    r.sig[0] = val(sa); r.sig[1] = val(sb); r.sig[2] = val(sc);
    S det = sa * sc - sb * sb;
    if (!(val(det) > 0.0)) { r.cull = std::isfinite(val(det)) ? CULL_DET : CULL_NONFINITE; return r; }
    r.A = sc / det; r.B = -sb / det; r.C = sa / det;

    // projected centre; pixel (i, j) has its centre at (i + 1/2, j + 1/2)
    r.u = vw.fx * p[0] / p[2] + vw.cx;
    r.v = vw.fy * p[1] / p[2] + vw.cy;

    // view-dependent colour from SH: rgb = sum_lm Y_lm(dir) k_lm + 1/2, clamped at 0
    S dvec[3] = {mean[0] - vw.campos[0], mean[1] - vw.campos[1], mean[2] - vw.campos[2]};
    S dn = sqrt(dvec[0] * dvec[0] + dvec[1] * dvec[1] + dvec[2] * dvec[2]);
    S Y[16];
    sh_basis<S>(st.sh_degree, dvec[0] / dn, dvec[1] / dn, dvec[2] / dn, Y);
    int K = (st.sh_degree + 1) * (st.sh_degree + 1);
    for (int c = 0; c < 3; ++c) {
        S acc(0.5);
        for (int k = 0; k < K; ++k) acc = acc + Y[k] * sh[3 * k + c];
        if (val(acc) < 0.0) { r.rgb[c] = S(0.0); r.clamp |= (uint8_t)(1u << c); }
        else r.rgb[c] = acc;
    }
    r.o = opac;
    r.beta = beta;

    // footprint: alpha >= alpha_min  <=>  q <= (ln(o/alpha_min)/kappa)^(2/beta)
    double o = val(opac), bt = val(beta);
    bool finite = std::isfinite(val(r.u)) && std::isfinite(val(r.v)) && std::isfinite(val(r.A)) &&
                  std::isfinite(val(r.B)) && std::isfinite(val(r.C)) && std::isfinite(o) && std::isfinite(bt) &&
                  std::isfinite(val(r.rgb[0])) && std::isfinite(val(r.rgb[1])) && std::isfinite(val(r.rgb[2]));
    if (!finite) { r.cull = CULL_NONFINITE; return r; }
    if (o < st.alpha_min) { r.cull = CULL_OPACITY; return r; }
    double L = std::log(o / st.alpha_min) / st.kappa;
    r.qmax = std::pow(L, 2.0 / bt) * (1.0 + std::ldexp(1.0, -10));
    double rx = std::sqrt(r.qmax * val(sa)), ry = std::sqrt(r.qmax * val(sc));
    double uu = val(r.u), vv = val(r.v);
    r.edges[0] = uu - rx - 0.5; r.edges[1] = uu + rx - 0.5;
    r.edges[2] = vv - ry - 0.5; r.edges[3] = vv + ry - 0.5;
    double fx0 = std::ceil(r.edges[0]), fx1 = std::floor(r.edges[1]);
    double fy0 = std::ceil(r.edges[2]), fy1 = std::floor(r.edges[3]);
    fx0 = std::max(fx0, 0.0); fy0 = std::max(fy0, 0.0);
    fx1 = std::min(fx1, (double)(vw.W - 1)); fy1 = std::min(fy1, (double)(vw.H - 1));
    if (!(fx0 <= fx1 && fy0 <= fy1)) { r.cull = CULL_EMPTY; return r; }
    r.pix[0] = (int)fx0; r.pix[1] = (int)fy0; r.pix[2] = (int)fx1; r.pix[3] = (int)fy1;
    r.tiles[0] = r.pix[0] / st.tile_w; r.tiles[1] = r.pix[1] / st.tile_h;
    r.tiles[2] = r.pix[2] / st.tile_w; r.tiles[3] = r.pix[3] / st.tile_h;
    r.touched = (uint32_t)((r.tiles[2] - r.tiles[0] + 1) * (r.tiles[3] - r.tiles[1] + 1));
    return r;
}

// ---------------------------------------------------------- compositing
// One fragment of a pixel's list: the splat's screen-space record.
struct Rec {
    double u, v, A, B, C, o, beta, qmax, r, g, b;
};

inline Rec load_rec(const double* rec, long idx) {
    const double* a = rec + 11 * idx;
    return Rec{a[0], a[1], a[2], a[3], a[4], a[5], a[6], a[7], a[8], a[9], a[10]};
}

// Falloff of Eq. (3) at pixel centre (px, py): G = exp(-kappa q^(beta/2)).
struct Frag { double dx, dy, q, P, G, oG, alpha; };

inline Frag eval_frag(const Rec& s, double px, double py, const Settings& st) {
    Frag f;
    f.dx = px - s.u;
    f.dy = py - s.v;
    f.q = s.A * f.dx * f.dx + 2.0 * s.B * f.dx * f.dy + s.C * f.dy * f.dy;
    if (f.q < 0.0) f.q = 0.0;
    f.P = (f.q > 0.0) ? std::pow(f.q, 0.5 * s.beta) : 0.0;
    f.G = std::exp(-st.kappa * f.P);
    f.oG = s.o * f.G;
    f.alpha = std::min(st.alpha_max, f.oG);
    return f;
}

// Unit roundoff of float32 (the precision of the rasterizer under test).
constexpr double U32 = 1.0 / 16777216.0;

// Per-pair bounds on how far a float32 projection's record may lie from the
// FP64 one (end-to-end comparisons; see orc_record_err_bound): centre error in
// pixels (u and v each), relative error of q from the conic, relative error
// of qmax.  Null when both sides use the same float32 records.
struct PairErr { double centre, conic, qmax; };

inline PairErr load_err(const double* perr, long idx) {
    if (!perr) return PairErr{0.0, 0.0, 0.0};
    const double* a = perr + 3 * idx;
    return PairErr{a[0], a[1], a[2]};
}

// Shear of the conic factor, |L10| / L11 = |B| / sqrt(AC - B^2): it multiplies
// the rounding error of L00 dx + L10 dy in a float32 evaluation of q.
inline double conic_shear(const Rec& s) {
    double det = s.A * s.C - s.B * s.B;
    return det > 0.0 ? std::fabs(s.B) / std::sqrt(det) : 0.0;
}

// First-order bound on |d ln(o G)| of a float32 evaluation of a fragment that
// takes the steps dx = px - u, dy = py - v, t = L00 dx + L10 dy (one fma),
// w = L11 dy, q = t^2 + w^2 (one fma), P = exp2((beta/2) log2 q),
// G = exp2(-kappa log2(e) P), o G, with correctly rounded + - * (unit
// roundoff u = 2^-24) and 1-ulp log2 / exp2:
//   |dq/q|     <= u (12 + 8 s),  s the conic shear;
//   |dP/P|     <= 2u + (beta/2) |dq/q| + 3 ln2 u |log2 P|;
//   |d ln oG|  <= 3u + kappa P (|dP/P| + 2u).
// End to end the record itself may differ from the FP64 one (PairErr), which
// adds kappa P (beta/2) (conic + 2 sqrt(2) centre |C d| / q) with C d the
// gradient of q / 2 at the pixel.  band_scale multiplies the result.
inline double frag_band(const Frag& f, const Rec& s, const Settings& st, const PairErr& e) {
    const double hb = 0.5 * s.beta;
    const double kP = st.kappa * f.P;
    const double dq = U32 * (12.0 + 8.0 * conic_shear(s));
    double dq_rec = 0.0;
    if (e.centre > 0.0 || e.conic > 0.0) {
        double gx = s.A * f.dx + s.B * f.dy, gy = s.B * f.dx + s.C * f.dy;
        double g = std::sqrt(gx * gx + gy * gy);
        dq_rec = e.conic + (f.q > 0.0 ? 2.0 * std::sqrt(2.0) * e.centre * g / f.q : 0.0);
    }
    const double lp = f.P > 0.0 ? std::fabs(std::log2(f.P)) : 0.0;
    const double dP = 2.0 * U32 + hb * (dq + dq_rec) + 3.0 * std::log(2.0) * U32 * lp;
    return st.band_scale * (3.0 * U32 + kP * (dP + 2.0 * U32));
}

// A decision is within the float32 band when its threshold lies within
// `band` of the FP64 value in log space.
inline bool near_log(double a, double b, double band) { return a > 0.0 && std::fabs(std::log(a / b)) <= band; }

struct PixelOut {
    double C[3];
    double D, A;  // extended channels: sum alpha T z and sum alpha T (zero background)
    double T;
    uint32_t n_contrib, n_listed, n_hit;
    uint8_t ambig;     // bit0 a skip decision (alpha vs alpha_min) within its band, bit1 o G within the band
                       // of alpha_max, bit2 a termination decision (T' vs t_min) within its band
    uint8_t n_branch;  // decisions within their band met along the path (saturates at 255)
    long last;         // record index of the last composited fragment (-1 if none): unlike n_contrib it
                       // does not depend on entries that no pixel of the tile composites
};

// One explicit list entry of a composited fragment (used by the adjoint).
struct Hit { long idx; long row; double alpha, T, z; Frag f; };

// Front-to-back compositing of one pixel over `list` (indices into rec, in
// order).  Skips fragments with alpha < alpha_min; stops before compositing a
// fragment that would take T below t_min.  n_contrib is the 1-based list
// position of the last composited fragment.
//
// Decision paths.  A skip or termination decision whose threshold lies within
// the fragment's float32 band (frag_band; the transmittance band accumulates
// alpha / (1 - alpha) times each composited fragment's band plus 2u per
// product) has two correct outcomes.  Such decisions are numbered in the order
// they are met; bit i of `path` set takes the other outcome at decision i
// (bits beyond 31 are 0).  path = 0 is the plain FP64 result.  The cap
// decision (o G vs alpha_max) only flags bit1: its two outcomes give the same
// alpha to within the band, so it is not enumerated.
//
// Extended channels (the depth maps of the mesh-extraction passage, Sec. 3.3):
// depth and opacity composited like a colour channel over a zero background,
// D = sum_k alpha_k T_k z_k and A = sum_k alpha_k T_k, with z the splat's
// camera-space depth (`depth`, nullable: z = 0).
template <class ListFn>
PixelOut composite_pixel(long count, ListFn idx_at, const double* rec, double px, double py, const Settings& st,
                         std::vector<Hit>* hits, const long* rows = nullptr, const double* depth = nullptr,
                         const double* perr = nullptr, uint32_t path = 0) {
    PixelOut o{{0, 0, 0}, 0.0, 0.0, 1.0, 0, 0, 0, 0, 0, -1};
    double T = 1.0;
    double tband = 0.0;  // bound on |d ln T| of the float32 transmittance
    int nb = 0;
    auto branch = [&](bool decision) {
        bool flip = nb < 32 && ((path >> nb) & 1u);
        if (nb < 255) ++nb;
        return flip ? !decision : decision;
    };
    for (long k = 0; k < count; ++k) {
        long idx = idx_at(k);
        Rec s = load_rec(rec, idx);
        Frag f = eval_frag(s, px, py, st);
        o.n_listed++;
        const double band = frag_band(f, s, st, load_err(perr, idx));
        bool skip = f.alpha < st.alpha_min;
        if (near_log(f.oG, st.alpha_min, band)) { o.ambig |= 1; skip = branch(skip); }
        if (near_log(f.oG, st.alpha_max, band)) o.ambig |= 2;
        if (skip) continue;
        o.n_hit++;
        const double Tn = T * (1.0 - f.alpha);
        const double tnext_band =
            tband + band * f.alpha / std::max(1.0 - f.alpha, 1e-12) + st.band_scale * 2.0 * U32;
        bool stop = Tn < st.t_min;
        if (near_log(Tn, st.t_min, tnext_band)) { o.ambig |= 4; stop = branch(stop); }
        if (stop) break;
        o.C[0] += s.r * f.alpha * T;
        o.C[1] += s.g * f.alpha * T;
        o.C[2] += s.b * f.alpha * T;
        const double z = depth ? depth[idx] : 0.0;
        o.D += z * f.alpha * T;
        o.A += f.alpha * T;
        if (hits) hits->push_back(Hit{idx, rows ? rows[k] : idx, f.alpha, T, z, f});
        T = Tn;
        tband = tnext_band;
        o.n_contrib = (uint32_t)(k + 1);
        o.last = idx;
    }
    for (int c = 0; c < 3; ++c) o.C[c] += T * st.bg[c];
    o.T = T;
    o.n_branch = (uint8_t)nb;
    return o;
}

// Adjoint of composite_pixel for one pixel, from its explicit hit list.
// g = dL/dC (3 values), gD = dL/dD, gA = dL/dA; writes into grad2d rows (11 per
// splat-view index): du, dv, dA, dB, dC, dopacity, dbeta, dr, dg, db, dz.
// Every channel c with fragment values c_k and background b gives
// dL/dalpha_k = T_k (c_k - B_k) g_c, where B_k is the channel composited
// behind fragment k per unit T_{k+1} (B = alpha_k c_k + (1 - alpha_k) B moving
// front-wards from B = b); depth has c_k = z_k, opacity c_k = 1, both b = 0.
void pixel_adjoint(const std::vector<Hit>& hits, double Tfinal, const double* g, double gD, double gA,
                   const double* rec, const Settings& st, double* grad2d) {
    double Bk[3] = {st.bg[0], st.bg[1], st.bg[2]};  // colour behind fragment k, per unit T_{k+1}
    double BD = 0.0, BA = 0.0;                       // depth and opacity behind fragment k
    (void)Tfinal;
    for (long k = (long)hits.size() - 1; k >= 0; --k) {
        const Hit& h = hits[k];
        Rec s = load_rec(rec, h.idx);
        double* gr = grad2d + 11 * h.row;
        double col[3] = {s.r, s.g, s.b};
        double dL_dalpha = 0.0;
        for (int c = 0; c < 3; ++c) {
            gr[7 + c] += h.alpha * h.T * g[c];
            dL_dalpha += h.T * (col[c] - Bk[c]) * g[c];
        }
        gr[10] += h.alpha * h.T * gD;
        dL_dalpha += h.T * (h.z - BD) * gD + h.T * (1.0 - BA) * gA;
        for (int c = 0; c < 3; ++c) Bk[c] = h.alpha * col[c] + (1.0 - h.alpha) * Bk[c];
        BD = h.alpha * h.z + (1.0 - h.alpha) * BD;
        BA = h.alpha + (1.0 - h.alpha) * BA;
        const Frag& f = h.f;
        if (f.oG > st.alpha_max) continue;  // alpha clamped: no dependence on o or G
        gr[5] += dL_dalpha * f.G;
        double dL_dG = dL_dalpha * s.o;
        double dG_dq = 0.0, dG_dbeta = 0.0;
        if (f.q > 0.0) {
            dG_dq = -st.kappa * f.G * (0.5 * s.beta) * f.P / f.q;
            dG_dbeta = -st.kappa * f.G * f.P * 0.5 * std::log(f.q);
        }
        double dL_dq = dL_dG * dG_dq;
        gr[6] += dL_dG * dG_dbeta;
        gr[0] += dL_dq * (-2.0 * (s.A * f.dx + s.B * f.dy));
        gr[1] += dL_dq * (-2.0 * (s.B * f.dx + s.C * f.dy));
        gr[2] += dL_dq * f.dx * f.dx;
        gr[3] += dL_dq * 2.0 * f.dx * f.dy;
        gr[4] += dL_dq * f.dy * f.dy;
    }
}

// ----------------------------------------------------------------- binning
// Smallest value of the footprint quadratic q(dx, dy) = A dx^2 + 2 B dx dy +
// C dy^2 (positive definite) over the box [x0, x1] x [y0, y1] of offsets from
// the centre.  q is convex: its minimum is 0 when the box holds the centre and
// otherwise lies on an edge, where q is a 1-D convex quadratic whose minimum
// is its vertex clamped into the edge.
double box_min_q(double A, double B, double C, double x0, double x1, double y0, double y1) {
    if (x0 <= 0.0 && 0.0 <= x1 && y0 <= 0.0 && 0.0 <= y1) return 0.0;
    auto q = [&](double x, double y) { return A * x * x + 2.0 * B * x * y + C * y * y; };
    auto clampd = [](double x, double lo, double hi) { return x < lo ? lo : (x > hi ? hi : x); };
    double best = HUGE_VAL;
    for (double xe : {x0, x1}) best = std::min(best, q(xe, clampd(-B * xe / C, y0, y1)));
    for (double ye : {y0, y1}) best = std::min(best, q(clampd(-B * ye / A, x0, x1), ye));
    return best;
}

// Which tiles list a pair.  The method only needs every tile holding a pixel
// centre with alpha >= alpha_min (q <= qmax) to list the splat; the footprint
// rule used here lists a tile of the pair's tile rectangle when the ellipse
// {q <= Q}, Q = qmax (1 + 2^-8), meets the tile's closed square
// [tx tw, (tx + 1) tw] x [ty th, (ty + 1) th] in pixel coordinates, i.e. when
// the minimum of q over the square is <= Q.  The margin 2^-8 keeps every
// decision that matters for the image (pixel centres lie half a pixel inside
// their tile, where q > qmax means alpha < alpha_min) far from the rule's
// boundary.
inline double tile_min_q(const Rec& s, int tx, int ty, int tw, int th, double grow) {
    return box_min_q(s.A, s.B, s.C, (double)tx * tw - s.u - grow, (double)(tx + 1) * tw - s.u + grow,
                     (double)ty * th - s.v - grow, (double)(ty + 1) * th - s.v + grow);
}
inline double footprint_Q(const Rec& s) { return s.qmax * (1.0 + std::ldexp(1.0, -8)); }
inline bool tile_listed(const Rec& s, int tx, int ty, int tw, int th) {
    return tile_min_q(s, tx, ty, tw, th, 0.0) <= footprint_Q(s);
}

// Float32 band of the tile rule.  A float32 implementation that derives each
// tile row's column interval from the record -- band edges ty th - v and
// (ty + 1) th - v, the ellipse's x-extent over the band from sqrt(Q),
// sqrt(Q - (L11 dy)^2), L10 dy and a quotient by L00, then u + extent -- is
// the exact rule for a square moved by at most `eps` pixels and a bound moved
// by a relative `eta`, with (unit roundoff u = 2^-24, correctly rounded
// operations; s the conic shear |L10| / L11):
//   eps = 2u (max(W, H) + |u| + |v|) + 32 u            (the two coordinate sums)
//   eta = u (16 + 8 s)                                 (the extent in q)
// plus, end to end, the record's own error: the centre bound adds to eps, the
// conic and qmax bounds to eta.  A decision is within the band when neither
// outcome is certain: the square grown by eps meets {q <= Q (1 + eta)} and the
// square shrunk by eps misses {q <= Q (1 - eta)}.
struct TileBand { double eps, eta; };

inline TileBand tile_band_params(const Rec& s, const View& w, const PairErr& e) {
    TileBand b;
    b.eps = 2.0 * U32 * ((double)std::max(w.W, w.H) + std::fabs(s.u) + std::fabs(s.v)) + 32.0 * U32 + e.centre;
    b.eta = U32 * (16.0 + 8.0 * conic_shear(s)) + e.conic + e.qmax;
    return b;
}

// 0: listed with certainty, 1: within the band, 2: not listed with certainty
// (the rectangle is not checked here).
inline int tile_status(const Rec& s, int tx, int ty, int tw, int th, const TileBand& b) {
    const double Q = footprint_Q(s);
    const double lo = tile_min_q(s, tx, ty, tw, th, b.eps);   // grown square
    const double hi = tile_min_q(s, tx, ty, tw, th, -b.eps);  // shrunk square
    if (lo > Q * (1.0 + b.eta)) return 2;
    if (hi <= Q * (1.0 - b.eta)) return 0;
    return 1;
}

int nthreads() {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
int thread_id() {
#ifdef _OPENMP
    return omp_get_thread_num();
#else
    return 0;
#endif
}

}  // namespace

extern "C" {

// Number of threads the oracle's parallel loops use.
int orc_num_threads(void) { return nthreads(); }
void orc_set_num_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

// Projection of N splats into V views (FP64).
//   views: V x 24 doubles: W, H, fx, fy, cx, cy, R[9] row-major, t[3], campos[3], pad
//   settings: kappa, rho, alpha_min, alpha_max, t_min, blur, znear, clip_fac, bg[3],
//             tile_w, tile_h, sh_degree, ambig (0 = 1e-5), ambig_pos, ambig_conic
// Outputs are [V][N]-indexed (view-major):
//   rec[11]: u, v, A, B, C, opacity, beta, qmax, r, g, b;  depth; z32 = RN_fp32(depth);
//   sigma2d[3] = (a, b, c) of Sigma'; edges[4] = u-rx-1/2, u+rx-1/2, v-ry-1/2, v+ry-1/2;
//   pix_rect[4] / tile_rect[4] inclusive (x0, y0, x1, y1); tiles_touched; cull; clamp.
int orc_project(int N, int V, const double* means, const double* scales, const double* quats, const double* opac,
                const double* betas, const double* sh, const double* views, const double* settings, double* rec,
                double* depth, float* z32, double* sigma2d, double* edges, int32_t* pix_rect, int32_t* tile_rect,
                uint32_t* tiles_touched, uint8_t* cull, uint8_t* clamp) {
    Settings st = read_settings(settings);
    std::vector<View> vw = read_views(views, V, st.tile_w, st.tile_h);
    int K = (st.sh_degree + 1) * (st.sh_degree + 1);
#pragma omp parallel for schedule(static)
    for (long i = 0; i < N; ++i) {
        double m[3], s[3], q[4];
        for (int a = 0; a < 3; ++a) { m[a] = means[3 * i + a]; s[a] = scales[3 * i + a]; }
        for (int a = 0; a < 4; ++a) q[a] = quats[4 * i + a];
        for (int v = 0; v < V; ++v) {
            Proj<double> p = project_one<double>(m, s, q, (double)opac[i], (double)betas[i], sh + (long)i * K * 3, vw[v], st);
            long o = (long)v * N + i;
            double r11[11] = {p.u, p.v, p.A, p.B, p.C, p.o, p.beta, p.qmax, p.rgb[0], p.rgb[1], p.rgb[2]};
            if (p.cull != KEEP) std::fill(r11, r11 + 11, 0.0);
            std::memcpy(rec + 11 * o, r11, sizeof r11);
            depth[o] = p.depth;
            z32[o] = (float)p.depth;
            for (int a = 0; a < 3; ++a) sigma2d[3 * o + a] = p.sig[a];
            for (int a = 0; a < 4; ++a) {
                edges[4 * o + a] = p.edges[a];
                pix_rect[4 * o + a] = p.pix[a];
                tile_rect[4 * o + a] = p.tiles[a];
            }
            tiles_touched[o] = p.cull == KEEP ? p.touched : 0;
            cull[o] = p.cull;
            clamp[o] = p.clamp;
        }
    }
    return 0;
}

// A-priori bounds on the error of a float32 projection record, per (view,
// splat) (perr, [V*N][3]): [0] centre, in pixels, for each of u and v; [1]
// relative error of q due to the conic, in the worst direction; [2] relative
// error of qmax.  First order in u = 2^-24, for a float32 projection that
// takes these steps (correctly rounded + - * / sqrt, 1-ulp exp and log):
//  * R from the normalised quaternion: entries within 8u (absolute);
//  * phi(beta) s: within 6u relative;
//  * T = J W: each entry within 4u of the sum of its two terms' magnitudes;
//  * U = T M with M = R diag(phi s): each entry within 3u sum_a |T_ia M_ab|;
//  * Sigma' = U U^T + blur I: a and c within 4u relative, b within
//    3u sum_k |U0k U1k|;
//  * det(Sigma') from non-negative terms, |x|^2 + blur (a0 + c0) + blur^2 with
//    x_k = (prod_{j != k} phi s_j) (R^T (T0 x T1))_k: R's error enters x
//    directly, the cross products within 8u of their terms' magnitudes, the
//    products of two scales within 13u; det's relative error is q's;
//  * the Cholesky factor of the conic: each entry within 4u relative, which
//    moves q by 4u (4 + 4 s) relative (s the conic shear).
// A perturbation dSigma' of Sigma' moves q by at most rho(Sigma'^-1 dSigma')
// relative (spectral radius); the conic bound sums these first-order effects.
// Centre: u = fx (x / z) + cx from a compensated camera-space centre, within
// 1/2 ulp(u) + 3u |u - cx| (v likewise; the larger is reported).  qmax =
// (ln(o / alpha_min) / kappa)^(2/beta) (1 + 2^-10) through log, log2 and exp2:
// within u (4 + (2/beta)(4 + 1 / ln(o / alpha_min)) + 3 |log2 qmax|).
// Culled pairs get zeros.
static double rho2(const double Si[3], const double X[3]) {
    // spectral radius of Si X for symmetric 2x2 Si = (s00, s01, s11), X = (x00, x01, x11)
    const double m00 = Si[0] * X[0] + Si[1] * X[1], m01 = Si[0] * X[1] + Si[1] * X[2];
    const double m10 = Si[1] * X[0] + Si[2] * X[1], m11 = Si[1] * X[1] + Si[2] * X[2];
    const double tr = 0.5 * (m00 + m11), dt = m00 * m11 - m01 * m10;
    const double disc = std::sqrt(std::max(tr * tr - dt, 0.0));
    return std::max(std::fabs(tr + disc), std::fabs(tr - disc));
}
static double ulp32(double x) {
    int e;
    std::frexp(std::fabs(x), &e);
    return std::ldexp(1.0, std::max(e, -125) - 24);
}

int orc_record_err_bound(int N, int V, const double* means, const double* scales, const double* quats,
                         const double* opac, const double* betas, const double* views, const double* settings,
                         double* perr) {
    Settings st = read_settings(settings);
    std::vector<View> vw = read_views(views, V, st.tile_w, st.tile_h);
    const double u = U32;
#pragma omp parallel for schedule(static)
    for (long i = 0; i < N; ++i) {
        const double* q4 = quats + 4 * i;
        const double qn = std::sqrt(q4[0] * q4[0] + q4[1] * q4[1] + q4[2] * q4[2] + q4[3] * q4[3]);
        const double w = q4[0] / qn, x = q4[1] / qn, y = q4[2] / qn, z = q4[3] / qn;
        const double R[9] = {1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y),
                             2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x),
                             2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)};
        const double phi = 2.0 / (1.0 + std::exp(-st.rho * (betas[i] - 2.0)));
        double ps[3], M[9];
        for (int b = 0; b < 3; ++b) ps[b] = phi * scales[3 * i + b];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) M[3 * a + b] = R[3 * a + b] * ps[b];
        const double o = opac[i], bt = betas[i];
        const double lnx = std::log(o / st.alpha_min);
        const double qmax = lnx > 0.0 ? std::pow(lnx / st.kappa, 2.0 / bt) * (1.0 + std::ldexp(1.0, -10)) : 0.0;
        const double e_qmax =
            lnx > 0.0 ? u * (4.0 + (2.0 / bt) * (4.0 + 1.0 / lnx) + 3.0 * std::fabs(std::log2(qmax))) : 0.0;
        for (int v = 0; v < V; ++v) {
            const View& c = vw[v];
            double* out = perr + 3 * ((long)v * N + i);
            out[0] = out[1] = out[2] = 0.0;
            double p[3];
            for (int a = 0; a < 3; ++a)
                p[a] = c.R[3 * a] * means[3 * i] + c.R[3 * a + 1] * means[3 * i + 1] + c.R[3 * a + 2] * means[3 * i + 2] +
                       c.t[a];
            if (!(p[2] > st.znear)) continue;
            const double limx = st.clip_fac * c.W / (2.0 * c.fx), limy = st.clip_fac * c.H / (2.0 * c.fy);
            const double xt = std::max(-limx, std::min(limx, p[0] / p[2])) * p[2];
            const double yt = std::max(-limy, std::min(limy, p[1] / p[2])) * p[2];
            const double J[6] = {c.fx / p[2], 0.0, -c.fx * xt / (p[2] * p[2]), 0.0, c.fy / p[2],
                                 -c.fy * yt / (p[2] * p[2])};
            double T[6], Tabs[6];
            for (int r = 0; r < 2; ++r)
                for (int b = 0; b < 3; ++b) {
                    T[3 * r + b] = J[3 * r] * c.R[b] + J[3 * r + 1] * c.R[3 + b] + J[3 * r + 2] * c.R[6 + b];
                    Tabs[3 * r + b] = std::fabs(J[3 * r] * c.R[b]) + std::fabs(J[3 * r + 1] * c.R[3 + b]) +
                                      std::fabs(J[3 * r + 2] * c.R[6 + b]);
                }
            double U[6], TM[6];  // U = T M (2 x 3) and sum_a |T_ia M_ab|
            for (int r = 0; r < 2; ++r)
                for (int b = 0; b < 3; ++b) {
                    U[3 * r + b] = T[3 * r] * M[b] + T[3 * r + 1] * M[3 + b] + T[3 * r + 2] * M[6 + b];
                    TM[3 * r + b] = std::fabs(T[3 * r] * M[b]) + std::fabs(T[3 * r + 1] * M[3 + b]) +
                                    std::fabs(T[3 * r + 2] * M[6 + b]);
                }
            const double a0 = U[0] * U[0] + U[1] * U[1] + U[2] * U[2];
            const double c0 = U[3] * U[3] + U[4] * U[4] + U[5] * U[5];
            const double sb = U[0] * U[3] + U[1] * U[4] + U[2] * U[5];
            const double sa = a0 + st.blur, sc = c0 + st.blur;
            const double det = sa * sc - sb * sb;
            if (!(det > 0.0) || !std::isfinite(det)) continue;
            const double Si[3] = {sc / det, -sb / det, sa / det};  // Sigma'^-1
            auto sym = [](const double a[2], const double b[2], double X[3]) {
                X[0] = 2.0 * a[0] * b[0];
                X[1] = a[0] * b[1] + a[1] * b[0];
                X[2] = 2.0 * a[1] * b[1];
            };
            double X[3], conic = 0.0;
            // rotation entries (absolute 8u): dM_ab = dR_ab ps_b moves column b of U by T[:, a]
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) {
                    const double ta[2] = {T[a], T[3 + a]}, ub[2] = {U[b], U[3 + b]};
                    sym(ta, ub, X);
                    conic += 8.0 * u * ps[b] * rho2(Si, X);
                }
            // T entries (4u of their terms): dT_ia moves row i of U by dT_ia M[a, :]
            for (int r = 0; r < 2; ++r)
                for (int a = 0; a < 3; ++a) {
                    const double g[2] = {U[0] * M[3 * a] + U[1] * M[3 * a + 1] + U[2] * M[3 * a + 2],
                                         U[3] * M[3 * a] + U[4] * M[3 * a + 1] + U[5] * M[3 * a + 2]};
                    const double e[2] = {r == 0 ? 1.0 : 0.0, r == 1 ? 1.0 : 0.0};
                    sym(e, g, X);
                    conic += 4.0 * u * Tabs[3 * r + a] * rho2(Si, X);
                }
            // U entries (3u of their terms) and phi s (6u relative, column b of U scaled)
            double u_terms = 0.0;
            for (int b = 0; b < 3; ++b) {
                const double ub[2] = {U[b], U[3 + b]};
                for (int r = 0; r < 2; ++r) {
                    const double e[2] = {r == 0 ? 1.0 : 0.0, r == 1 ? 1.0 : 0.0};
                    sym(e, ub, X);
                    conic += 3.0 * u * TM[3 * r + b] * rho2(Si, X);
                    u_terms += std::fabs(U[3 * r + b]) * TM[3 * r + b];
                }
                sym(ub, ub, X);
                conic += 6.0 * u * rho2(Si, X);
            }
            // Sigma' entries: a, c relative 4u; b absolute 3u sum |U0k U1k|
            const double babs = std::fabs(U[0] * U[3]) + std::fabs(U[1] * U[4]) + std::fabs(U[2] * U[5]);
            conic += 4.0 * u * (sa * Si[0] + sc * Si[2]);
            conic += 3.0 * u * babs * (std::fabs(Si[1]) + std::sqrt(Si[0] * Si[2]));
            // det from the non-negative terms
            const double n[3] = {T[1] * T[5] - T[2] * T[4], T[2] * T[3] - T[0] * T[5], T[0] * T[4] - T[1] * T[3]};
            const double nT[3] = {Tabs[1] * Tabs[5] + Tabs[2] * Tabs[4], Tabs[2] * Tabs[3] + Tabs[0] * Tabs[5],
                                  Tabs[0] * Tabs[4] + Tabs[1] * Tabs[3]};
            const double n1 = std::fabs(n[0]) + std::fabs(n[1]) + std::fabs(n[2]);
            const double pp[3] = {ps[1] * ps[2], ps[0] * ps[2], ps[0] * ps[1]};
            double ddet = 3.0 * u * det + st.blur * (4.0 * u * (a0 + c0) + 6.0 * u * u_terms);
            for (int k = 0; k < 3; ++k) {
                double mk = 0.0, dm = 8.0 * u * n1;
                for (int j = 0; j < 3; ++j) {
                    mk += R[3 * j + k] * n[j];
                    dm += std::fabs(R[3 * j + k]) * (8.0 * u * nT[j]) + 3.0 * u * std::fabs(R[3 * j + k] * n[j]);
                }
                const double xk = pp[k] * mk;
                ddet += 2.0 * std::fabs(xk) * (13.0 * u * std::fabs(xk) + pp[k] * dm);
            }
            conic += ddet / det;
            // the stored Cholesky factor
            const double shear = std::fabs(sb) / std::sqrt(det);
            conic += 4.0 * u * (4.0 + 4.0 * shear);
            const double uu = c.fx * p[0] / p[2] + c.cx, vv = c.fy * p[1] / p[2] + c.cy;
            // (+ 2^-40 of the magnitudes: the FP64 reference's own rounding)
            out[0] = std::max(0.5 * ulp32(uu) + 3.0 * u * std::fabs(uu - c.cx),
                              0.5 * ulp32(vv) + 3.0 * u * std::fabs(vv - c.cy)) +
                     std::ldexp(std::fabs(uu) + std::fabs(vv) + c.cx + c.cy, -40);
            out[1] = conic;
            out[2] = e_qmax;
        }
    }
    return 0;
}

uint64_t orc_bin_count(long VN, const uint32_t* tiles_touched) {
    uint64_t m = 0;
    for (long k = 0; k < VN; ++k) m += tiles_touched[k];
    return m;
}

long orc_total_tiles(int V, const double* views, int tile_w, int tile_h) {
    std::vector<View> vw = read_views(views, V, tile_w, tile_h);
    return vw.back().tile_base + (long)vw.back().tiles_x * vw.back().tiles_y;
}

// Binning: one instance per (view, splat, listed tile) -- a tile of the pair's
// tile rectangle whose square meets the footprint ellipse (tile_listed) --
// emitted in (view, splat, tile-row, tile-column) order with key =
// tile << 32 | bits(z32) and value = view * N + splat; stable sort by key;
// ranges[t] = [first, end) of tile t in the sorted list ((0, 0) when empty).
// rec: [V*N][11] records (u, v, A, B, C, opacity, beta, qmax, r, g, b).
long orc_bin(int N, int V, const int32_t* tile_rect, const uint32_t* tiles_touched, const uint32_t* zbits,
             const double* views, int tile_w, int tile_h, const double* rec, uint64_t* keys, uint32_t* vals,
             uint32_t* ranges) {
    std::vector<View> vw = read_views(views, V, tile_w, tile_h);
    long T = vw.back().tile_base + (long)vw.back().tiles_x * vw.back().tiles_y;
    // a view's keys lie in its own tile range, so each view is sorted on its
    // own and the views are concatenated in order
    std::vector<std::vector<std::pair<uint64_t, uint32_t>>> inst(V);
#pragma omp parallel for schedule(dynamic, 1)
    for (int v = 0; v < V; ++v) {
        for (long i = 0; i < N; ++i) {
            long o = (long)v * N + i;
            if (tiles_touched[o] == 0) continue;
            const int32_t* r = tile_rect + 4 * o;
            const Rec s = load_rec(rec, o);
            for (int ty = r[1]; ty <= r[3]; ++ty)
                for (int tx = r[0]; tx <= r[2]; ++tx) {
                    if (!tile_listed(s, tx, ty, tile_w, tile_h)) continue;
                    uint64_t tile = (uint64_t)(vw[v].tile_base + (long)ty * vw[v].tiles_x + tx);
                    inst[v].emplace_back((tile << 32) | zbits[o], (uint32_t)o);
                }
        }
        std::stable_sort(inst[v].begin(), inst[v].end(),
                         [](const std::pair<uint64_t, uint32_t>& a, const std::pair<uint64_t, uint32_t>& b) {
                             return a.first < b.first;
                         });
    }
    for (long t = 0; t < T; ++t) { ranges[2 * t] = 0; ranges[2 * t + 1] = 0; }
    size_t k = 0;
    for (int v = 0; v < V; ++v) {
        for (const auto& e : inst[v]) {
            keys[k] = e.first;
            vals[k] = e.second;
            uint64_t t = e.first >> 32;
            if (k == 0 || (keys[k - 1] >> 32) != t) ranges[2 * t] = (uint32_t)k;
            ranges[2 * t + 1] = (uint32_t)(k + 1);
            ++k;
        }
        std::vector<std::pair<uint64_t, uint32_t>>().swap(inst[v]);
    }
    return (long)k;
}

// Per pair: the tiles of its rectangle listed with certainty (n_in) and those
// whose decision lies within the float32 band (n_band) -- see tile_status;
// perr ([V*N][3], nullable) adds the end-to-end record error bounds.
int orc_bin_pair_counts(int N, int V, const double* views, int tile_w, int tile_h, const int32_t* tile_rect,
                        const uint32_t* tiles_touched, const double* rec, const double* perr, uint32_t* n_in,
                        uint32_t* n_band) {
    std::vector<View> vw = read_views(views, V, tile_w, tile_h);
    const long VN = (long)V * N;
#pragma omp parallel for schedule(dynamic, 4096)
    for (long o = 0; o < VN; ++o) {
        uint32_t a = 0, b = 0;
        if (tiles_touched[o] != 0) {
            const int32_t* r = tile_rect + 4 * o;
            const Rec s = load_rec(rec, o);
            const TileBand tb = tile_band_params(s, vw[o / N], load_err(perr, o));
            for (int ty = r[1]; ty <= r[3]; ++ty)
                for (int tx = r[0]; tx <= r[2]; ++tx) {
                    int st = tile_status(s, tx, ty, tile_w, tile_h, tb);
                    a += st == 0;
                    b += st == 1;
                }
        }
        n_in[o] = a;
        n_band[o] = b;
    }
    return 0;
}

// The (pair, global tile) decisions of every rectangle that lie within the
// float32 band, in (view, splat, row, column) order, with the FP64 rule's
// outcome (listed 1/0).  Writes at most `cap`; returns the total count.
long orc_bin_band(int N, int V, const double* views, int tile_w, int tile_h, const int32_t* tile_rect,
                  const uint32_t* tiles_touched, const double* rec, const double* perr, long cap, uint32_t* pair,
                  uint32_t* tile, uint8_t* listed) {
    std::vector<View> vw = read_views(views, V, tile_w, tile_h);
    long n = 0;
    for (int v = 0; v < V; ++v)
        for (long i = 0; i < N; ++i) {
            long o = (long)v * N + i;
            if (tiles_touched[o] == 0) continue;
            const int32_t* r = tile_rect + 4 * o;
            const Rec s = load_rec(rec, o);
            const TileBand tb = tile_band_params(s, vw[v], load_err(perr, o));
            for (int ty = r[1]; ty <= r[3]; ++ty)
                for (int tx = r[0]; tx <= r[2]; ++tx) {
                    if (tile_status(s, tx, ty, tile_w, tile_h, tb) != 1) continue;
                    if (n < cap) {
                        pair[n] = (uint32_t)o;
                        tile[n] = (uint32_t)(vw[v].tile_base + (long)ty * vw[v].tiles_x + tx);
                        listed[n] = tile_listed(s, tx, ty, tile_w, tile_h) ? 1 : 0;
                    }
                    ++n;
                }
        }
    return n;
}

// Status of L listed instances (pair vals[k], global tile tiles[k]) under the
// tile rule: 0 listed with certainty, 1 within the band, 2 not listed with
// certainty, 3 a tile outside the pair's view or rectangle.
int orc_instance_status(int N, int V, const double* views, int tile_w, int tile_h, const int32_t* tile_rect,
                        const double* rec, const double* perr, long L, const uint32_t* vals, const uint32_t* tiles,
                        uint8_t* status) {
    std::vector<View> vw = read_views(views, V, tile_w, tile_h);
#pragma omp parallel for schedule(static)
    for (long k = 0; k < L; ++k) {
        const long o = vals[k];
        const int v = (int)(o / N);
        const View& w = vw[v];
        const long lt = (long)tiles[k] - w.tile_base;
        uint8_t st = 3;
        if (lt >= 0 && lt < (long)w.tiles_x * w.tiles_y) {
            const int tx = (int)(lt % w.tiles_x), ty = (int)(lt / w.tiles_x);
            const int32_t* r = tile_rect + 4 * o;
            if (tx >= r[0] && tx <= r[2] && ty >= r[1] && ty <= r[3]) {
                const Rec s = load_rec(rec, o);
                st = (uint8_t)tile_status(s, tx, ty, tile_w, tile_h, tile_band_params(s, w, load_err(perr, o)));
            }
        }
        status[k] = st;
    }
    return 0;
}

// Tiled forward: every pixel composites the sorted list of its tile.
// Outputs (concatenated over views): image [3][H][W] per view, final_T,
// n_contrib, n_listed, n_hit, ambig, n_branch and last (see PixelOut); with `depth`
// ([V*N] splat depths) non-null, the extended channels out_depth and
// out_alpha ([P] each, nullable).  perr ([V*N][3], nullable): end-to-end
// record error bounds that widen the decision bands; paths ([P], nullable):
// the decision path of each pixel (composite_pixel; null = 0 everywhere).
int orc_render_fwd(int N, int V, const double* views, const double* settings, const double* rec,
                   const uint32_t* vals, const uint32_t* ranges, const double* perr, const uint32_t* paths,
                   double* image, double* final_T, uint32_t* n_contrib, uint32_t* n_listed, uint32_t* n_hit,
                   uint8_t* ambig, uint8_t* n_branch, int64_t* last, const double* depth, double* out_depth,
                   double* out_alpha) {
    (void)N;
    Settings st = read_settings(settings);
    std::vector<View> vw = read_views(views, V, st.tile_w, st.tile_h);
    for (int v = 0; v < V; ++v) {
        const View& w = vw[v];
#pragma omp parallel for schedule(dynamic, 4)
        for (long y = 0; y < w.H; ++y)
            for (long x = 0; x < w.W; ++x) {
                long t = w.tile_base + (y / st.tile_h) * w.tiles_x + x / st.tile_w;
                uint32_t s0 = ranges[2 * t], s1 = ranges[2 * t + 1];
                long p = w.pix_base + y * w.W + x;
                PixelOut po = composite_pixel(
                    (long)s1 - s0, [&](long k) { return (long)vals[s0 + k]; }, rec, x + 0.5, y + 0.5, st, nullptr,
                    nullptr, depth, perr, paths ? paths[p] : 0u);
                long HW = (long)w.W * w.H;
                for (int c = 0; c < 3; ++c) image[3 * w.pix_base + c * HW + y * w.W + x] = po.C[c];
                final_T[p] = po.T;
                n_contrib[p] = po.n_contrib;
                if (out_depth) out_depth[p] = po.D;
                if (out_alpha) out_alpha[p] = po.A;
                if (n_listed) n_listed[p] = po.n_listed;
                if (n_hit) n_hit[p] = po.n_hit;
                if (ambig) ambig[p] = po.ambig;
                if (n_branch) n_branch[p] = po.n_branch;
                if (last) last[p] = po.last;
            }
    }
    return 0;
}

// o G of n fragments (record rec[k] at pixel centre (px[k], py[k])) and the
// float32 band of ln(o G) (frag_band; perr [n][3] nullable).
int orc_fragment_band(long n, const double* rec, const double* px, const double* py, const double* settings,
                      const double* perr, double* oG, double* band) {
    Settings st = read_settings(settings);
#pragma omp parallel for schedule(static)
    for (long k = 0; k < n; ++k) {
        const Rec s = load_rec(rec, k);
        const Frag f = eval_frag(s, px[k], py[k], st);
        oG[k] = f.oG;
        band[k] = frag_band(f, s, st, load_err(perr, k));
    }
    return 0;
}

// Which of a pixel's correct results a float32 rasterizer produced.  Every
// pixel whose plain FP64 composite meets a decision within its band has
// several correct results, one per decision path; they are enumerated depth
// first (at most max_leaves) and the path whose result matches the given one
// -- the same last composited fragment (g_last: record index, -1 if none), the
// same n_hit and n_listed when given (g_nlisted entries of 0xFFFFFFFF are not
// compared: n_listed counts list entries, so it is compared only where both
// sides built the same list), every colour channel within
// tol_view[v] and final T within tol_T -- is chosen (the closest match when
// several do).  Outputs per pixel: paths (0 unless status 1) and status:
//   0  no decision within its band: one correct result (path 0);
//   1  resolved: the given result is the one of `paths`;
//   2  o G within the band of alpha_max (the cap's two outcomes give the
//      same image but different derivatives, so it cannot be told apart);
//   3  more than max_leaves paths;
//   4  no path's result matches.
// The given result only selects among results the oracle computes itself.
int orc_resolve(int N, int V, const double* views, const double* settings, const double* rec, const uint32_t* vals,
                const uint32_t* ranges, const double* perr, const float* g_image, const float* g_T,
                const int64_t* g_last, const uint32_t* g_nhit, const uint32_t* g_nlisted, const double* tol_view,
                double tol_T, int max_leaves, uint32_t* paths, uint8_t* status) {
    (void)N;
    Settings st = read_settings(settings);
    std::vector<View> vw = read_views(views, V, st.tile_w, st.tile_h);
    for (int v = 0; v < V; ++v) {
        const View& w = vw[v];
        const long HW = (long)w.W * w.H;
#pragma omp parallel for schedule(dynamic, 16)
        for (long y = 0; y < w.H; ++y)
            for (long x = 0; x < w.W; ++x) {
                const long t = w.tile_base + (y / st.tile_h) * w.tiles_x + x / st.tile_w;
                const uint32_t s0 = ranges[2 * t], s1 = ranges[2 * t + 1];
                const long p = w.pix_base + y * w.W + x;
                auto run = [&](uint32_t path) {
                    return composite_pixel((long)s1 - s0, [&](long k) { return (long)vals[s0 + k]; }, rec, x + 0.5,
                                           y + 0.5, st, nullptr, nullptr, nullptr, perr, path);
                };
                auto mismatch = [&](const PixelOut& o) {  // < 0: outputs differ; else the largest error
                    if (o.last != g_last[p]) return -1.0;
                    if (g_nhit && o.n_hit != g_nhit[p]) return -1.0;
                    if (g_nlisted && g_nlisted[p] != 0xFFFFFFFFu && o.n_listed != g_nlisted[p]) return -1.0;
                    double e = 0.0;
                    for (int c = 0; c < 3; ++c)
                        e = std::max(e, std::fabs(o.C[c] - (double)g_image[3 * w.pix_base + c * HW + y * w.W + x]));
                    if (e > tol_view[v] || std::fabs(o.T - (double)g_T[p]) > tol_T) return -1.0;
                    return e;
                };
                const PixelOut o0 = run(0u);
                paths[p] = 0u;
                if (o0.ambig & 2) { status[p] = 2; continue; }
                if (o0.n_branch == 0) { status[p] = 0; continue; }
                // depth-first enumeration: explore(prefix, j0) yields the path
                // `prefix`, then for each decision j >= j0 met along it the paths
                // that agree with it before j and flip decision j
                int leaves = 0;
                bool overflow = false;
                double best = -1.0;
                uint32_t best_path = 0u;
                std::vector<std::pair<uint32_t, int>> stack{{0u, 0}};
                while (!stack.empty()) {
                    auto [prefix, j0] = stack.back();
                    stack.pop_back();
                    if (++leaves > max_leaves) { overflow = true; break; }
                    const PixelOut o = prefix ? run(prefix) : o0;
                    const double e = mismatch(o);
                    if (e >= 0.0 && (best < 0.0 || e < best)) { best = e; best_path = prefix; }
                    for (int j = std::min<int>(o.n_branch, 32) - 1; j >= j0; --j)
                        stack.emplace_back(prefix | (1u << j), j + 1);
                }
                if (overflow) status[p] = 3;
                else if (best < 0.0) status[p] = 4;
                else { status[p] = 1; paths[p] = best_path; }
            }
    }
    return 0;
}

// Candidate lists per view for the brute-force renderer: every non-culled
// splat of the view, ordered by (z32, splat index).
static std::vector<std::vector<long>> depth_order(int N, int V, const uint32_t* zbits, const uint8_t* cull) {
    std::vector<std::vector<long>> ord(V);
    for (int v = 0; v < V; ++v) {
        for (long i = 0; i < N; ++i)
            if (cull[(long)v * N + i] == KEEP) ord[v].push_back((long)v * N + i);
        std::stable_sort(ord[v].begin(), ord[v].end(), [&](long a, long b) { return zbits[a] < zbits[b]; });
    }
    return ord;
}

// Brute force: each pixel composites every non-culled splat of its view in
// (z32, index) order.  With pix_rect non-null, splats whose pixel rectangle
// misses the pixel are left out (used for fast window evaluation).  window
// (V x 4: x0, y0, x1, y1 inclusive; nullable) restricts the pixels evaluated;
// pixels outside it are left untouched.
int orc_brute_fwd(int N, int V, const double* views, const double* settings, const double* rec,
                  const uint32_t* zbits, const uint8_t* cull, const int32_t* pix_rect, const int32_t* window,
                  double* image, double* final_T, uint32_t* n_hit, uint8_t* ambig) {
    Settings st = read_settings(settings);
    std::vector<View> vw = read_views(views, V, st.tile_w, st.tile_h);
    auto ord = depth_order(N, V, zbits, cull);
    for (int v = 0; v < V; ++v) {
        const View& w = vw[v];
        int x0 = 0, y0 = 0, x1 = w.W - 1, y1 = w.H - 1;
        if (window) { x0 = std::max(x0, window[4 * v]); y0 = std::max(y0, window[4 * v + 1]);
                      x1 = std::min(x1, window[4 * v + 2]); y1 = std::min(y1, window[4 * v + 3]); }
        std::vector<long> cand;
        for (long o : ord[v]) {
            if (pix_rect) {
                const int32_t* r = pix_rect + 4 * o;
                if (r[2] < x0 || r[0] > x1 || r[3] < y0 || r[1] > y1) continue;
            }
            cand.push_back(o);
        }
#pragma omp parallel for schedule(dynamic, 1)
        for (long y = y0; y <= y1; ++y) {
            std::vector<long> list;
            for (long x = x0; x <= x1; ++x) {
                list.clear();
                for (long o : cand) {
                    if (pix_rect) {
                        const int32_t* r = pix_rect + 4 * o;
                        if (x < r[0] || x > r[2] || y < r[1] || y > r[3]) continue;
                    }
                    list.push_back(o);
                }
                PixelOut po = composite_pixel((long)list.size(), [&](long k) { return list[k]; }, rec, x + 0.5,
                                              y + 0.5, st, nullptr);
                long p = w.pix_base + y * w.W + x;
                long HW = (long)w.W * w.H;
                for (int c = 0; c < 3; ++c) image[3 * w.pix_base + c * HW + y * w.W + x] = po.C[c];
                final_T[p] = po.T;
                if (n_hit) n_hit[p] = po.n_hit;
                if (ambig) ambig[p] = po.ambig;
            }
        }
    }
    return 0;
}

// Render adjoint over the tiled lists: re-runs the forward per pixel keeping
// the explicit list of composited fragments (alpha_k, T_k) and back-propagates
// dL/dimage (and, with `depth` non-null, dL/ddepth and dL/dalpha of the
// extended channels, each nullable) into grad2d [V*N][11] (du, dv, dA, dB, dC,
// dopacity, dbeta, dr, dg, db, dz).  Accumulation uses one buffer per thread,
// summed in thread order.
int orc_render_bwd(int N, int V, const double* views, const double* settings, const double* rec,
                   const uint32_t* vals, const uint32_t* ranges, const double* perr, const uint32_t* paths,
                   const double* dL_dimage, const double* depth, const double* dL_ddepth, const double* dL_dalpha,
                   double* grad2d) {
    Settings st = read_settings(settings);
    std::vector<View> vw = read_views(views, V, st.tile_w, st.tile_h);
    long VN = (long)V * N;
    int nt = nthreads();
    std::vector<std::vector<double>> acc(nt);
#pragma omp parallel
    {
        std::vector<double>& g2 = acc[thread_id()];
        g2.assign(11 * VN, 0.0);
        std::vector<Hit> hits;
        for (int v = 0; v < V; ++v) {
            const View& w = vw[v];
            long HW = (long)w.W * w.H;
#pragma omp for schedule(dynamic, 4)
            for (long y = 0; y < w.H; ++y)
                for (long x = 0; x < w.W; ++x) {
                    long t = w.tile_base + (y / st.tile_h) * w.tiles_x + x / st.tile_w;
                    uint32_t s0 = ranges[2 * t], s1 = ranges[2 * t + 1];
                    hits.clear();
                    const long p = w.pix_base + y * w.W + x;
                    PixelOut po = composite_pixel(
                        (long)s1 - s0, [&](long k) { return (long)vals[s0 + k]; }, rec, x + 0.5, y + 0.5, st, &hits,
                        nullptr, depth, perr, paths ? paths[p] : 0u);
                    double g[3];
                    for (int c = 0; c < 3; ++c) g[c] = dL_dimage[3 * w.pix_base + c * HW + y * w.W + x];
                    const double gD = (depth && dL_ddepth) ? dL_ddepth[p] : 0.0;
                    const double gA = (depth && dL_dalpha) ? dL_dalpha[p] : 0.0;
                    pixel_adjoint(hits, po.T, g, gD, gA, rec, st, g2.data());
                }
        }
    }
    std::fill(grad2d, grad2d + 11 * VN, 0.0);
    for (int k = 0; k < nt; ++k)
        if (!acc[k].empty())
            for (long j = 0; j < 11 * VN; ++j) grad2d[j] += acc[k][j];
    return 0;
}

// Window forward + adjoint by brute force with the pixel-rectangle filter:
// pixels in window (V x 4, inclusive) only.  Returns sum over the window of
// dL_dimage . image (+ dL_ddepth . D + dL_dalpha . A of the extended channels
// when `depth` is non-null) in *loss and, for the `n_watch` splat-view indices
// in `watch`, their grad2d rows (n_watch x 11).  `decisions` receives a hash of
// every skip/terminate/clamp decision taken (for finite-difference checks).
int orc_window_fwdbwd(int N, int V, const double* views, const double* settings, const double* rec,
                      const uint32_t* zbits, const uint8_t* cull, const int32_t* pix_rect, const int32_t* window,
                      const double* dL_dimage, const double* depth, const double* dL_ddepth,
                      const double* dL_dalpha, int n_watch, const long* watch, double* loss, double* watch_grad,
                      uint64_t* decisions) {
    Settings st = read_settings(settings);
    std::vector<View> vw = read_views(views, V, st.tile_w, st.tile_h);
    auto ord = depth_order(N, V, zbits, cull);
    // watched index -> output row
    std::vector<std::pair<long, int>> wmap;
    for (int k = 0; k < n_watch; ++k) wmap.emplace_back(watch[k], k);
    std::sort(wmap.begin(), wmap.end());
    double total = 0.0;
    uint64_t dh = 1469598103934665603ull;
    std::fill(watch_grad, watch_grad + 11 * (long)n_watch, 0.0);
    for (int v = 0; v < V; ++v) {
        const View& w = vw[v];
        int x0 = std::max(0, window[4 * v]), y0 = std::max(0, window[4 * v + 1]);
        int x1 = std::min(w.W - 1, window[4 * v + 2]), y1 = std::min(w.H - 1, window[4 * v + 3]);
        if (x0 > x1 || y0 > y1) continue;
        std::vector<long> cand;
        for (long o : ord[v]) {
            const int32_t* r = pix_rect + 4 * o;
            if (r[2] < x0 || r[0] > x1 || r[3] < y0 || r[1] > y1) continue;
            cand.push_back(o);
        }
        long HW = (long)w.W * w.H;
        std::vector<long> list, rows;
        std::vector<Hit> hits;
        // gradients accumulate in a compact buffer with one row per candidate
        std::vector<double> g2(11 * cand.size(), 0.0);
        for (long y = y0; y <= y1; ++y)
            for (long x = x0; x <= x1; ++x) {
                list.clear();
                rows.clear();
                for (size_t c = 0; c < cand.size(); ++c) {
                    const int32_t* r = pix_rect + 4 * cand[c];
                    if (x < r[0] || x > r[2] || y < r[1] || y > r[3]) continue;
                    list.push_back(cand[c]);
                    rows.push_back((long)c);
                }
                hits.clear();
                PixelOut po = composite_pixel((long)list.size(), [&](long k) { return list[k]; }, rec, x + 0.5,
                                              y + 0.5, st, &hits, rows.data(), depth);
                double g[3];
                for (int c = 0; c < 3; ++c) {
                    g[c] = dL_dimage[3 * w.pix_base + c * HW + y * w.W + x];
                    total += g[c] * po.C[c];
                }
                const long p = w.pix_base + y * w.W + x;
                const double gD = (depth && dL_ddepth) ? dL_ddepth[p] : 0.0;
                const double gA = (depth && dL_dalpha) ? dL_dalpha[p] : 0.0;
                total += gD * po.D + gA * po.A;
                pixel_adjoint(hits, po.T, g, gD, gA, rec, st, g2.data());
                for (const Hit& h : hits) {
                    uint64_t e = (uint64_t)h.idx * 1315423911ull + (uint64_t)(h.f.oG > st.alpha_max);
                    dh = (dh ^ e) * 1099511628211ull;
                }
                dh = (dh ^ (uint64_t)po.n_contrib) * 1099511628211ull;
            }
        for (auto& pr : wmap) {
            auto it = std::lower_bound(cand.begin(), cand.end(), pr.first);
            // cand is in depth order, not index order: search linearly on a miss
            long c = -1;
            if (it != cand.end() && *it == pr.first) c = it - cand.begin();
            else for (size_t j = 0; j < cand.size(); ++j) if (cand[j] == pr.first) { c = (long)j; break; }
            if (c < 0) continue;
            for (int j = 0; j < 11; ++j) watch_grad[11 * pr.second + j] += g2[11 * c + j];
        }
    }
    *loss = total;
    if (decisions) *decisions = dh;
    return 0;
}

// Projection adjoint: grad2d [V*N][11] -> gradients of the splat inputs,
// summed over views in ascending order.  The Jacobian of every projected
// quantity with respect to (mean, scale, quat, opacity, beta) comes from
// forward-mode dual numbers through project_one; the SH coefficients enter the
// colour linearly, so their gradient is Y_lm(dir) times the unclamped colour
// gradient.
int orc_project_bwd(int N, int V, const double* means, const double* scales, const double* quats, const double* opac,
                    const double* betas, const double* sh, const double* views, const double* settings,
                    const double* grad2d, double* g_means, double* g_scales, double* g_quats, double* g_opac,
                    double* g_betas, double* g_sh) {
    Settings st = read_settings(settings);
    std::vector<View> vw = read_views(views, V, st.tile_w, st.tile_h);
    int K = (st.sh_degree + 1) * (st.sh_degree + 1);
    typedef Dual<12> D;
#pragma omp parallel for schedule(static)
    for (long i = 0; i < N; ++i) {
        D m[3], s[3], q[4];
        for (int a = 0; a < 3; ++a) m[a] = D::var(means[3 * i + a], a);
        for (int a = 0; a < 3; ++a) s[a] = D::var(scales[3 * i + a], 3 + a);
        for (int a = 0; a < 4; ++a) q[a] = D::var(quats[4 * i + a], 6 + a);
        D o = D::var(opac[i], 10), b = D::var(betas[i], 11);
        double gacc[12] = {0};
        std::vector<double> gsh(3 * K, 0.0);
        for (int v = 0; v < V; ++v) {
            long idx = (long)v * N + i;
            Proj<D> p = project_one<D>(m, s, q, o, b, sh + (long)i * K * 3, vw[v], st);
            if (p.cull != KEEP) continue;
            const double* g = grad2d + 11 * idx;
            const D* outs[11] = {&p.u, &p.v, &p.A, &p.B, &p.C, &p.o, &p.beta, &p.rgb[0], &p.rgb[1], &p.rgb[2], &p.z};
            for (int k = 0; k < 12; ++k) {
                double acc = 0.0;
                for (int j = 0; j < 11; ++j) acc += g[j] * outs[j]->d[k];
                gacc[k] += acc;
            }
            // SH coefficients: d rgb_c / d k_lc = Y_lm(dir), zero on a clamped channel
            double dv[3] = {means[3 * i] - vw[v].campos[0], means[3 * i + 1] - vw[v].campos[1],
                            means[3 * i + 2] - vw[v].campos[2]};
            double dn = std::sqrt(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2]);
            double Y[16];
            sh_basis<double>(st.sh_degree, dv[0] / dn, dv[1] / dn, dv[2] / dn, Y);
            for (int c = 0; c < 3; ++c) {
                if (p.clamp & (1u << c)) continue;
                for (int k = 0; k < K; ++k) gsh[3 * k + c] += Y[k] * g[7 + c];
            }
        }
        for (int a = 0; a < 3; ++a) g_means[3 * i + a] = gacc[a];
        for (int a = 0; a < 3; ++a) g_scales[3 * i + a] = gacc[3 + a];
        for (int a = 0; a < 4; ++a) g_quats[4 * i + a] = gacc[6 + a];
        g_opac[i] = gacc[10];
        g_betas[i] = gacc[11];
        for (int k = 0; k < 3 * K; ++k) g_sh[(long)i * 3 * K + k] = gsh[k];
    }
    return 0;
}

// Level-set surface points along depth-map rays (Sec. 3.3, mesh extraction).
// Readings (the paper gives the procedure, not its constants or its choice of
// the distribution g):
//   * ray of pixel p of view v: from the camera centre through the pixel
//     centre, unit direction w; origin x0 = the depth-map point at distance
//     t0 = (D/A) |d_c| along w (D, A the extended channels, d_c the camera-space
//     direction with unit z, so t0 w has camera depth D/A); rays with
//     A < min_alpha carry no surface;
//   * density (Eq. 9): d(x) = sum_i o_i exp(-kappa m_i(x)^beta_i), m_i the 3-D
//     Mahalanobis distance under Sigma_i = M_i M_i^T, M_i = R(q_i) diag(phi s_i)
//     (Eq. 4, 6), over the candidates of the pixel: the splats in its tile's
//     list whose screen footprint covers it (q <= qmax), since a splat outside
//     it has density below alpha_min-level on the ray;
//   * g = the candidate with the largest term o_i exp(-kappa m_i(x0)^beta_i)
//     (the dominating distribution g* of Eq. 10); sigma_g(w) = |M_g^T w|;
//   * K samples t_k = t0 + span sigma_g (2k/(K-1) - 1); the first k with
//     d_k < level <= d_{k+1} brackets the surface closest to the camera; t* by
//     linear interpolation; the normal is grad f / |grad f| with
//     f = s sqrt(-2 log d), i.e. -grad d / |grad d| at x0 + t* w.
// Outputs per ray: points [R][3], normals [R][3], valid [R], dominant [R]
// (pair index v*N + i of g, -1 if none), t_star [R] and margins [R][3]: the
// relative gap between the two largest terms at x0, min over the bracketing
// samples of |d_k - level| / level, and |A - min_alpha| (decision margins).
static void surface_M(const double* scale, const double* quat, double beta, const Settings& st, double M[9]) {
    double qn = std::sqrt(quat[0] * quat[0] + quat[1] * quat[1] + quat[2] * quat[2] + quat[3] * quat[3]);
    double w = quat[0] / qn, x = quat[1] / qn, y = quat[2] / qn, z = quat[3] / qn;
    double Rq[9] = {1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y),
                    2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x),
                    2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)};
    double phi = 2.0 / (1.0 + std::exp(-st.rho * (beta - 2.0)));
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) M[3 * a + b] = Rq[3 * a + b] * phi * scale[b];
}

// o exp(-kappa m^beta) at x and (optionally) its gradient with respect to x.
static double surface_term(const double M[9], const double* mu, double o, double beta, const double x[3],
                           const Settings& st, double grad[3]) {
    // m^2 = |M^-1 (x - mu)|^2 with M = R diag(d): M^-1 = diag(1/d) R^T
    double dx[3] = {x[0] - mu[0], x[1] - mu[1], x[2] - mu[2]};
    double Minv[9];
    double det = M[0] * (M[4] * M[8] - M[5] * M[7]) - M[1] * (M[3] * M[8] - M[5] * M[6]) +
                 M[2] * (M[3] * M[7] - M[4] * M[6]);
    Minv[0] = (M[4] * M[8] - M[5] * M[7]) / det; Minv[1] = (M[2] * M[7] - M[1] * M[8]) / det;
    Minv[2] = (M[1] * M[5] - M[2] * M[4]) / det; Minv[3] = (M[5] * M[6] - M[3] * M[8]) / det;
    Minv[4] = (M[0] * M[8] - M[2] * M[6]) / det; Minv[5] = (M[2] * M[3] - M[0] * M[5]) / det;
    Minv[6] = (M[3] * M[7] - M[4] * M[6]) / det; Minv[7] = (M[1] * M[6] - M[0] * M[7]) / det;
    Minv[8] = (M[0] * M[4] - M[1] * M[3]) / det;
    double y[3];
    for (int a = 0; a < 3; ++a) y[a] = Minv[3 * a] * dx[0] + Minv[3 * a + 1] * dx[1] + Minv[3 * a + 2] * dx[2];
    double m2 = y[0] * y[0] + y[1] * y[1] + y[2] * y[2];
    double P = m2 > 0.0 ? std::pow(m2, 0.5 * beta) : 0.0;
    double val = o * std::exp(-st.kappa * P);
    if (grad) {
        // d/dx exp(-kappa (m^2)^(beta/2)) = -kappa (beta/2) (m^2)^(beta/2 - 1) 2 Minv^T y exp(...)
        double c = (m2 > 0.0) ? -st.kappa * beta * std::pow(m2, 0.5 * beta - 1.0) * val : 0.0;
        for (int a = 0; a < 3; ++a) grad[a] = c * (Minv[a] * y[0] + Minv[3 + a] * y[1] + Minv[6 + a] * y[2]);
    }
    return val;
}

int orc_surface_points(int N, int V, const double* means, const double* scales, const double* quats,
                       const double* opac, const double* betas, const double* views, const double* settings,
                       const double* rec, const uint32_t* vals, const uint32_t* ranges, const double* depth_map,
                       const double* alpha_map, const long* pixels, long R, int K, double level, double span,
                       double min_alpha, double* points, double* normals, int32_t* valid, long* dominant,
                       double* t_star, double* margins) {
    Settings st = read_settings(settings);
    std::vector<View> vw = read_views(views, V, st.tile_w, st.tile_h);
#pragma omp parallel for schedule(dynamic, 4)
    for (long r = 0; r < R; ++r) {
        for (int a = 0; a < 3; ++a) { points[3 * r + a] = 0.0; normals[3 * r + a] = 0.0; margins[3 * r + a] = 0.0; }
        valid[r] = 0;
        dominant[r] = -1;
        t_star[r] = 0.0;
        long p = pixels[r];
        int v = 0;
        while (v + 1 < V && vw[v + 1].pix_base <= p) ++v;
        const View& w = vw[v];
        long local = p - w.pix_base;
        int px = (int)(local % w.W), py = (int)(local / w.W);
        double A = alpha_map[p], D = depth_map[p];
        margins[3 * r + 2] = std::fabs(A - min_alpha);
        if (!(A >= min_alpha) || !(A > 0.0)) continue;
        // ray: camera-space direction with unit z, to world space by R^T
        double dc[3] = {(px + 0.5 - w.cx) / w.fx, (py + 0.5 - w.cy) / w.fy, 1.0};
        double nd = std::sqrt(dc[0] * dc[0] + dc[1] * dc[1] + 1.0);
        double wd[3];
        for (int a = 0; a < 3; ++a) wd[a] = (w.R[a] * dc[0] + w.R[3 + a] * dc[1] + w.R[6 + a] * dc[2]) / nd;
        double t0 = (D / A) * nd;
        // candidates: the tile's list entries whose screen footprint covers the pixel
        long t = w.tile_base + (py / st.tile_h) * w.tiles_x + px / st.tile_w;
        std::vector<long> cand;
        for (uint32_t k = ranges[2 * t]; k < ranges[2 * t + 1]; ++k) {
            long idx = vals[k];
            Rec s = load_rec(rec, idx);
            Frag f = eval_frag(s, px + 0.5, py + 0.5, st);
            if (f.q <= s.qmax) cand.push_back(idx);
        }
        if (cand.empty()) continue;
        std::vector<double> Ms(9 * cand.size());
        for (size_t c = 0; c < cand.size(); ++c) {
            long i = cand[c] % N;
            surface_M(scales + 3 * i, quats + 4 * i, betas[i], st, &Ms[9 * c]);
        }
        double x0[3] = {w.campos[0] + t0 * wd[0], w.campos[1] + t0 * wd[1], w.campos[2] + t0 * wd[2]};
        double best = -1.0, second = -1.0;
        long bc = -1;
        for (size_t c = 0; c < cand.size(); ++c) {
            long i = cand[c] % N;
            double val = surface_term(&Ms[9 * c], means + 3 * i, opac[i], betas[i], x0, st, nullptr);
            if (val > best) { second = best; best = val; bc = (long)c; }
            else if (val > second) second = val;
        }
        dominant[r] = cand[bc];
        margins[3 * r] = best > 0.0 ? (best - std::max(second, 0.0)) / best : 0.0;
        const double* Mg = &Ms[9 * bc];
        double sg = 0.0;
        for (int b = 0; b < 3; ++b) {
            double c = Mg[b] * wd[0] + Mg[3 + b] * wd[1] + Mg[6 + b] * wd[2];  // (M^T w)_b
            sg += c * c;
        }
        sg = std::sqrt(sg);
        std::vector<double> tk(K), dk(K, 0.0);
        for (int k = 0; k < K; ++k) {
            tk[k] = t0 + span * sg * (2.0 * k / (K - 1) - 1.0);
            double x[3] = {w.campos[0] + tk[k] * wd[0], w.campos[1] + tk[k] * wd[1], w.campos[2] + tk[k] * wd[2]};
            for (size_t c = 0; c < cand.size(); ++c) {
                long i = cand[c] % N;
                dk[k] += surface_term(&Ms[9 * c], means + 3 * i, opac[i], betas[i], x, st, nullptr);
            }
        }
        int kc = -1;
        for (int k = 0; k + 1 < K; ++k)
            if (dk[k] < level && dk[k + 1] >= level) { kc = k; break; }
        if (kc < 0) continue;
        double mg = std::fabs(dk[kc] - level);
        mg = std::min(mg, std::fabs(dk[kc + 1] - level));
        for (int k = 0; k < kc; ++k) mg = std::min(mg, std::fabs(dk[k] - level));
        margins[3 * r + 1] = mg / level;
        double ts = tk[kc] + (level - dk[kc]) / (dk[kc + 1] - dk[kc]) * (tk[kc + 1] - tk[kc]);
        double xs[3] = {w.campos[0] + ts * wd[0], w.campos[1] + ts * wd[1], w.campos[2] + ts * wd[2]};
        double gd[3] = {0.0, 0.0, 0.0};
        for (size_t c = 0; c < cand.size(); ++c) {
            long i = cand[c] % N;
            double g3[3];
            surface_term(&Ms[9 * c], means + 3 * i, opac[i], betas[i], xs, st, g3);
            for (int a = 0; a < 3; ++a) gd[a] += g3[a];
        }
        double gn = std::sqrt(gd[0] * gd[0] + gd[1] * gd[1] + gd[2] * gd[2]);
        if (!(gn > 0.0)) continue;
        for (int a = 0; a < 3; ++a) { points[3 * r + a] = xs[a]; normals[3 * r + a] = -gd[a] / gn; }
        t_star[r] = ts;
        valid[r] = 1;
    }
    return 0;
}

// Real SH basis (for tests): n directions (x, y, z) -> n x (deg+1)^2 values.
int orc_sh_basis(int degree, long n, const double* dirs, double* out) {
    int K = (degree + 1) * (degree + 1);
    for (long i = 0; i < n; ++i) sh_basis<double>(degree, dirs[3 * i], dirs[3 * i + 1], dirs[3 * i + 2], out + K * i);
    return 0;
}

}  // extern "C"

// ------------------------------------------------ surface regulariser (GSR)
// Sec. 3.3, Eq. (9)-(13), with the neighbour lists of Sec. 4.2 (16 nearest
// centres, refreshed periodically).  Readings (the paper leaves these open):
//   * Neighbourhood N(j) of splat j: j itself in slot 0, then its K - 1
//     nearest other centres by (squared distance, index).
//   * Sample set X: one point per (selected) splat, x_j = mu_j + M_j xi_j with
//     M = R diag(phi s) (Eq. 4, 6) and xi_j given (standard normal draws made
//     by the caller), so x depends on splat j's parameters.
//   * d(x) of Eq. (9) sums o_i exp(-kappa m_i^beta_i) over N(j) (kappa = 1/2
//     is the printed 1/2, m_i the Mahalanobis distance under M_i).
//   * g* is the neighbour with the largest term at x; its normal n is the
//     rotation column of its smallest scale, s_min = phi s of that axis.
//   * Eq. (10) with s_min^beta (the falloff of Eq. 9 along the normal of a
//     flat splat of opacity 1): dbar = exp(-kappa (|h| / s_min)^beta*),
//     h = <x - mu_g*, n>; equal to the printed form at beta = 2.
//   * Eq. (11): f = sigma s_min sqrt(-ln d / kappa) (the printed -2 log d at
//     kappa = 1/2), sigma = sign(h) (+1 at 0) for both f and fbar; d is
//     floored at 1e-30 and -ln d clamped at 0 (f = 0 where d >= 1).
//   * Eq. (12): l_sdf = |fbar - f|.  Eq. (13): l_nor = |grad f / |grad f| - n|^2
//     with grad f / |grad f| = -sigma grad d / |grad d|; 0 unless d and
//     |grad d| both exceed 1e-30 (below that the SDF or its direction is
//     undefined in float32).
//   * The loss of a sample is w_sdf l_sdf + w_nor l_nor; its gradient is the
//     exact derivative with every discrete choice (N(j), g*, its axis, sigma,
//     the clamps) held fixed.
// Parity: pinned by brute-force neighbour lists, closed forms of lone and
// paired splats and central differences of the loss.
namespace {

template <int D> Dual<D> log(const Dual<D>& a) {
    Dual<D> r(std::log(a.v)); for (int k = 0; k < D; ++k) r.d[k] = a.d[k] / a.v; return r;
}
using std::log;
template <class S> S powS(const S& a, const S& b) { return exp(b * log(a)); }
template <class S> S absS(const S& a) { return val(a) < 0.0 ? -a : a; }

constexpr double kGsrFloor = 1e-30;

struct GsrInfo {
    int gstar = 0, kstar = 0;
    // decision margins: g* (relative gap of the two largest terms), sigma
    // (|h| / |x - mu_g*|, the relative conditioning of h), the kink of
    // |fbar - f| (relative), the clamp at d = 1 (|ln d|), the normal axis
    // (relative gap of the two smallest scales), the conditioning of the
    // normal term (|grad d| / sum_i |grad T_i|: its direction is
    // ill-conditioned where the terms cancel), and the floors of d and
    // |grad d| (min of |ln(d / 1e-30)| and |ln(|grad d| / 1e-30)|)
    double margins[7] = {0, 0, 0, 0, 0, 0, 0};
};

template <class S>
void gsr_rot(const S q[4], S R[9]) {
    S qn = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    S w = q[0] / qn, x = q[1] / qn, y = q[2] / qn, z = q[3] / qn;
    R[0] = 1.0 - 2.0 * (y * y + z * z); R[1] = 2.0 * (x * y - w * z); R[2] = 2.0 * (x * z + w * y);
    R[3] = 2.0 * (x * y + w * z); R[4] = 1.0 - 2.0 * (x * x + z * z); R[5] = 2.0 * (y * z - w * x);
    R[6] = 2.0 * (x * z - w * y); R[7] = 2.0 * (y * z + w * x); R[8] = 1.0 - 2.0 * (x * x + y * y);
}

// Loss terms of one sample.  Parameter arrays hold the K neighbours in slot
// order (slot 0 = the sampled splat).
template <class S>
void gsr_sample(int K, const S (*mean)[3], const S (*scale)[3], const S (*quat)[4], const S* opac, const S* beta,
                const double xi[3], const Settings& st, S& l_sdf, S& l_nor, GsrInfo& info) {
    std::vector<std::array<S, 9>> R(K);
    std::vector<std::array<S, 3>> sig(K);
    for (int i = 0; i < K; ++i) {
        gsr_rot(quat[i], R[i].data());
        S phi = 2.0 / (1.0 + exp(-st.rho * (beta[i] - 2.0)));
        for (int k = 0; k < 3; ++k) sig[i][k] = phi * scale[i][k];
    }
    // the sample x = mu_0 + R_0 diag(sig_0) xi
    S x[3];
    for (int a = 0; a < 3; ++a) {
        x[a] = mean[0][a];
        for (int k = 0; k < 3; ++k) x[a] = x[a] + R[0][3 * a + k] * (sig[0][k] * xi[k]);
    }
    // Eq. (9) and its gradient in x
    S d(0.0), gd[3] = {S(0.0), S(0.0), S(0.0)};
    double best = -1.0, second = -1.0, gsum = 0.0;
    int gs = 0;
    for (int i = 0; i < K; ++i) {
        S dx[3] = {x[0] - mean[i][0], x[1] - mean[i][1], x[2] - mean[i][2]};
        S y[3];
        for (int k = 0; k < 3; ++k)
            y[k] = (R[i][k] * dx[0] + R[i][3 + k] * dx[1] + R[i][6 + k] * dx[2]) / sig[i][k];
        S q = y[0] * y[0] + y[1] * y[1] + y[2] * y[2];
        S T, c(0.0);
        if (val(q) > 0.0) {
            S P = powS(q, beta[i] * 0.5);
            T = opac[i] * exp(-st.kappa * P);
            c = -st.kappa * beta[i] * P / q * T;  // dT/dq * 2
        } else {
            T = opac[i];
        }
        d = d + T;
        double gi2 = 0.0;
        for (int a = 0; a < 3; ++a) {
            S ga = c * (R[i][3 * a] * y[0] / sig[i][0] + R[i][3 * a + 1] * y[1] / sig[i][1] +
                        R[i][3 * a + 2] * y[2] / sig[i][2]);
            gd[a] = gd[a] + ga;
            gi2 += val(ga) * val(ga);
        }
        gsum += std::sqrt(gi2);
        if (val(T) > best) { second = best; best = val(T); gs = i; }
        else if (val(T) > second) second = val(T);
    }
    info.gstar = gs;
    info.margins[0] = best > 0.0 ? (best - std::max(second, 0.0)) / best : 0.0;
    // normal and s_min of g*
    int ks = 0;
    for (int k = 1; k < 3; ++k) if (val(sig[gs][k]) < val(sig[gs][ks])) ks = k;
    double s2 = 1e300;
    for (int k = 0; k < 3; ++k) if (k != ks) s2 = std::min(s2, val(sig[gs][k]));
    info.kstar = ks;
    info.margins[4] = (s2 - val(sig[gs][ks])) / val(sig[gs][ks]);
    S n[3] = {R[gs][ks], R[gs][3 + ks], R[gs][6 + ks]};
    S smin = sig[gs][ks];
    S h = (x[0] - mean[gs][0]) * n[0] + (x[1] - mean[gs][1]) * n[1] + (x[2] - mean[gs][2]) * n[2];
    double sg = val(h) >= 0.0 ? 1.0 : -1.0;
    {
        double xm2 = 0.0;
        for (int a = 0; a < 3; ++a) xm2 += (val(x[a]) - val(mean[gs][a])) * (val(x[a]) - val(mean[gs][a]));
        info.margins[1] = xm2 > 0.0 ? std::fabs(val(h)) / std::sqrt(xm2) : 0.0;
    }
    S r = absS(h) / smin;
    S A = val(r) > 0.0 ? powS(r, beta[gs] * 0.5) : S(0.0);  // fbar / (sigma s_min)
    S Ld = val(d) > kGsrFloor ? -log(d) : S(-std::log(kGsrFloor));
    info.margins[3] = std::fabs(val(Ld));
    S B = val(Ld) > 0.0 ? sqrt(Ld / st.kappa) : S(0.0);  // f / (sigma s_min)
    S diff = A - B;
    info.margins[2] = std::fabs(val(diff)) / std::max(std::max(val(A), val(B)), 1e-300);
    l_sdf = smin * absS(diff);
    S g2 = gd[0] * gd[0] + gd[1] * gd[1] + gd[2] * gd[2];
    info.margins[5] = gsum > 0.0 ? std::sqrt(val(g2)) / gsum : 0.0;
    const double gabs = std::sqrt(val(g2));
    info.margins[6] = std::min(val(d) > 0.0 ? std::fabs(std::log(val(d) / kGsrFloor)) : 0.0,
                               gabs > 0.0 ? std::fabs(std::log(gabs / kGsrFloor)) : 0.0);
    // the normal term needs the SDF (d above its floor) and a direction
    if (val(d) > kGsrFloor && gabs > kGsrFloor) {
        S gn = sqrt(g2);
        l_nor = S(0.0);
        for (int a = 0; a < 3; ++a) {
            S e = -sg * gd[a] / gn - n[a];
            l_nor = l_nor + e * e;
        }
    } else {
        l_nor = S(0.0);
    }
}

}  // namespace

extern "C" {

// Neighbour lists: knn[j][0] = j, then the K - 1 nearest other centres by
// (squared distance, index) (brute force).
int orc_knn(int N, const double* means, int K, int32_t* knn) {
#pragma omp parallel for schedule(dynamic, 16)
    for (int j = 0; j < N; ++j) {
        std::vector<std::pair<double, int>> dist;
        dist.reserve(N);
        for (int i = 0; i < N; ++i) {
            if (i == j) continue;
            double dx = means[3 * i] - means[3 * j], dy = means[3 * i + 1] - means[3 * j + 1],
                   dz = means[3 * i + 2] - means[3 * j + 2];
            dist.emplace_back(dx * dx + dy * dy + dz * dz, i);
        }
        int m = std::min(K - 1, (int)dist.size());
        std::partial_sort(dist.begin(), dist.begin() + m, dist.end());
        knn[(long)j * K] = j;
        for (int s = 1; s < K; ++s) knn[(long)j * K + s] = s - 1 < m ? dist[s - 1].second : -1;
    }
    return 0;
}

// GSR losses and gradients.  knn [N][K] (slot 0 = j); xi [N][3]; mask [N]
// (nullable: every sample); per sample l_sdf, l_nor, gstar (neighbour slot),
// margins [N][7]; grads [N][12] (mean 3, scale 3, quat 4, opacity, beta) of
// sum_j mask_j (w_sdf l_sdf + w_nor l_nor), accumulated when non-null.
int orc_gsr(int N, const double* means, const double* scales, const double* quats, const double* opac,
            const double* betas, const double* settings, int K, const int32_t* knn, const double* xi,
            const uint8_t* mask, double w_sdf, double w_nor, double* l_sdf, double* l_nor, int32_t* gstar,
            double* margins, double* grads) {
    Settings st = read_settings(settings);
    int nt = nthreads();
    std::vector<std::vector<double>> tg(grads ? nt : 0, std::vector<double>(grads ? (size_t)N * 12 : 0, 0.0));
#pragma omp parallel for schedule(dynamic, 8)
    for (int j = 0; j < N; ++j) {
        l_sdf[j] = l_nor[j] = 0.0;
        gstar[j] = -1;
        for (int k = 0; k < 7; ++k) margins[7 * j + k] = 0.0;
        if (mask && !mask[j]) continue;
        const int32_t* nb = knn + (long)j * K;
        std::vector<double> mu(3 * K), sc(3 * K), qu(4 * K), op(K), be(K);
        for (int s = 0; s < K; ++s) {
            long i = nb[s];
            for (int a = 0; a < 3; ++a) { mu[3 * s + a] = means[3 * i + a]; sc[3 * s + a] = scales[3 * i + a]; }
            for (int a = 0; a < 4; ++a) qu[4 * s + a] = quats[4 * i + a];
            op[s] = opac[i];
            be[s] = betas[i];
        }
        GsrInfo info;
        double ls, ln;
        gsr_sample<double>(K, reinterpret_cast<const double(*)[3]>(mu.data()),
                           reinterpret_cast<const double(*)[3]>(sc.data()),
                           reinterpret_cast<const double(*)[4]>(qu.data()), op.data(), be.data(), xi + 3 * j, st, ls,
                           ln, info);
        l_sdf[j] = ls;
        l_nor[j] = ln;
        gstar[j] = info.gstar;
        for (int k = 0; k < 7; ++k) margins[7 * j + k] = info.margins[k];
        if (!grads) continue;
        double* g = tg[thread_id()].data();
        using D12 = Dual<12>;
        std::vector<D12> dm(3 * K), ds(3 * K), dq(4 * K), dop(K), db(K);
        for (int s = 0; s < K; ++s) {
            for (int a = 0; a < 3; ++a) { dm[3 * s + a] = D12(mu[3 * s + a]); ds[3 * s + a] = D12(sc[3 * s + a]); }
            for (int a = 0; a < 4; ++a) dq[4 * s + a] = D12(qu[4 * s + a]);
            dop[s] = D12(op[s]);
            db[s] = D12(be[s]);
        }
        for (int s = 0; s < K; ++s) {
            // seed neighbour s's twelve parameters
            for (int a = 0; a < 3; ++a) { dm[3 * s + a].d[a] = 1.0; ds[3 * s + a].d[3 + a] = 1.0; }
            for (int a = 0; a < 4; ++a) dq[4 * s + a].d[6 + a] = 1.0;
            dop[s].d[10] = 1.0;
            db[s].d[11] = 1.0;
            GsrInfo di;
            D12 a_sdf, a_nor;
            gsr_sample<D12>(K, reinterpret_cast<const D12(*)[3]>(dm.data()),
                            reinterpret_cast<const D12(*)[3]>(ds.data()), reinterpret_cast<const D12(*)[4]>(dq.data()),
                            dop.data(), db.data(), xi + 3 * j, st, a_sdf, a_nor, di);
            long i = nb[s];
            for (int k = 0; k < 12; ++k) g[12 * i + k] += w_sdf * a_sdf.d[k] + w_nor * a_nor.d[k];
            for (int a = 0; a < 3; ++a) { dm[3 * s + a].d[a] = 0.0; ds[3 * s + a].d[3 + a] = 0.0; }
            for (int a = 0; a < 4; ++a) dq[4 * s + a].d[6 + a] = 0.0;
            dop[s].d[10] = 0.0;
            db[s].d[11] = 0.0;
        }
    }
    if (grads)
        for (int t = 0; t < nt; ++t)
            for (long k = 0; k < (long)N * 12; ++k) grads[k] += tg[t][k];
    return 0;
}

}  // extern "C"
