// project.hip -- per-Gaussian projection onto the ERP screen (forward) and
// its chain rule back to the Gaussian parameters (backward).
//
// Both kernels are one thread per Gaussian and bandwidth-bound (236 B of
// parameters in per Gaussian).  CDNA4 runs FP64 vector math at the FP32
// non-packed rate, so the whole projection is done in double precision at no
// measurable cost; only the 48-byte blend record is rounded to float.
//
// Forward (Sec. 3.2-3.3):
//   t = W m + t_cw                                   (Eq. 1)
//   lon = atan2(t_x, t_z), lat = asin(t_y / t_r)     (Eq. 3)
//   s = (lon / pi, 2 lat / pi), p = (s + 1) (W, H)/2  (Eq. 4, 5)
//   J = dp/dt                                        (Eq. 10-16)
//   Sigma2D = (J W) Sigma (J W)^T + dilation I        (Eq. 9)
// computed as V V^T with V = J W R(q) diag(S), which is exactly Eq. 9 for
// Sigma = R diag(S)^2 R^T and keeps the 2x2 covariance positive in floating
// point.  The radius of influence is the axis-aligned box of the
// alpha = alpha_min iso-ellipse; its pixel columns wrap across the seam.
//
// A pinhole camera (Eq. 2) replaces Eq. 3-5 and 10-16 by
// p = (f_x t_x / t_z + c_x, f_y t_y / t_z + c_y) and its Jacobian, taken at
// the direction t_x / t_z, t_y / t_z clamped to 1.3 times the image's angular
// half-extent around its middle (3DGS's guard against the affine
// approximation's blow-up near the image plane; the centre is not clamped),
// orders by t_z, culls t_z <= near_plane and clamps the box's columns to the
// image.
//
// Backward (Sec. 3.4, Eq. 18-20): from the per-Gaussian accumulators
// dL/dp, the exponent's second moments, dL/do, dL/drgb to dL/dm, dL/dS, dL/dq,
// dL/do, dL/dSH and dL/ds, through the replaced omnidirectional terms
// dSigma2D/dSigma, dJ/dt, dp/ds and ds/dt.
#include "internal.h"

#include <cmath>

namespace omnigs {
namespace {

constexpr double kPi = 3.141592653589793238462643383279502884;
constexpr double kLn2d = 0.693147180559945309417232121458176568;
constexpr double kInvPi = 0.318309886183790671537767526745028724;

// Real SH basis constants (Condon-Shortley phase, index l*l + l + m,
// z polar axis), from N_l^m = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!):
constexpr double kSH0 = 0.28209479177387814;   // 1 / (2 sqrt(pi))
constexpr double kSH1 = 0.48860251190291992;   // sqrt(3 / (4 pi))
constexpr double kSH2a = 1.0925484305920792;   // sqrt(15 / (4 pi))
constexpr double kSH2b = 0.31539156525252005;  // sqrt(5 / (16 pi))
constexpr double kSH2c = 0.54627421529603959;  // sqrt(15 / (16 pi))
constexpr double kSH3a = 0.59004358992664352;  // sqrt(35 / (32 pi))
constexpr double kSH3b = 2.8906114426405538;   // sqrt(105 / (4 pi))
constexpr double kSH3c = 0.45704579946446572;  // sqrt(21 / (32 pi))
constexpr double kSH3d = 0.37317633259011540;  // sqrt(7 / (16 pi))
constexpr double kSH3e = 1.4453057213202769;   // sqrt(105 / (16 pi))

template <int D>
__device__ inline void sh_basis(double x, double y, double z, double *Y) {
    Y[0] = kSH0;
    if (D >= 1) {
        Y[1] = -kSH1 * y;
        Y[2] = kSH1 * z;
        Y[3] = -kSH1 * x;
    }
    if (D >= 2) {
        const double xx = x * x, yy = y * y, zz = z * z;
        Y[4] = kSH2a * x * y;
        Y[5] = -kSH2a * y * z;
        Y[6] = kSH2b * (2.0 * zz - xx - yy);
        Y[7] = -kSH2a * x * z;
        Y[8] = kSH2c * (xx - yy);
        if (D >= 3) {
            Y[9] = -kSH3a * y * (3.0 * xx - yy);
            Y[10] = kSH3b * x * y * z;
            Y[11] = -kSH3c * y * (4.0 * zz - xx - yy);
            Y[12] = kSH3d * z * (2.0 * zz - 3.0 * xx - 3.0 * yy);
            Y[13] = -kSH3c * x * (4.0 * zz - xx - yy);
            Y[14] = kSH3e * z * (xx - yy);
            Y[15] = -kSH3a * x * (xx - 3.0 * yy);
        }
    }
}

// Gradient of basis polynomial k w.r.t. (x, y, z) (k constant after
// unrolling, so the switch folds).
__device__ inline void sh_basis_grad_k(int k, double x, double y, double z, double d[3]) {
    const double xx = x * x, yy = y * y, zz = z * z;
    switch (k) {
        case 1: d[0] = 0.0; d[1] = -kSH1; d[2] = 0.0; break;
        case 2: d[0] = 0.0; d[1] = 0.0; d[2] = kSH1; break;
        case 3: d[0] = -kSH1; d[1] = 0.0; d[2] = 0.0; break;
        case 4: d[0] = kSH2a * y; d[1] = kSH2a * x; d[2] = 0.0; break;
        case 5: d[0] = 0.0; d[1] = -kSH2a * z; d[2] = -kSH2a * y; break;
        case 6: d[0] = -2.0 * kSH2b * x; d[1] = -2.0 * kSH2b * y; d[2] = 4.0 * kSH2b * z; break;
        case 7: d[0] = -kSH2a * z; d[1] = 0.0; d[2] = -kSH2a * x; break;
        case 8: d[0] = 2.0 * kSH2c * x; d[1] = -2.0 * kSH2c * y; d[2] = 0.0; break;
        case 9: d[0] = -kSH3a * 6.0 * x * y; d[1] = -kSH3a * 3.0 * (xx - yy); d[2] = 0.0; break;
        case 10: d[0] = kSH3b * y * z; d[1] = kSH3b * x * z; d[2] = kSH3b * x * y; break;
        case 11:
            d[0] = kSH3c * 2.0 * x * y;
            d[1] = -kSH3c * (4.0 * zz - xx - 3.0 * yy);
            d[2] = -kSH3c * 8.0 * y * z;
            break;
        case 12:
            d[0] = -kSH3d * 6.0 * x * z;
            d[1] = -kSH3d * 6.0 * y * z;
            d[2] = kSH3d * (6.0 * zz - 3.0 * xx - 3.0 * yy);
            break;
        case 13:
            d[0] = -kSH3c * (4.0 * zz - 3.0 * xx - yy);
            d[1] = kSH3c * 2.0 * x * y;
            d[2] = -kSH3c * 8.0 * x * z;
            break;
        case 14: d[0] = kSH3e * 2.0 * x * z; d[1] = -kSH3e * 2.0 * y * z; d[2] = kSH3e * (xx - yy); break;
        case 15: d[0] = -kSH3a * 3.0 * (xx - yy); d[1] = kSH3a * 6.0 * x * y; d[2] = 0.0; break;
        default: d[0] = d[1] = d[2] = 0.0; break;  // k = 0: constant
    }
}

// Everything the forward computes for one Gaussian, in double precision.
struct Proj {
    double t[3], tr, rho;
    double depth;  // sort key: t_r (ERP) or t_z (pinhole)
    double px, py;
    double J[6];   // Jacobian of the projection used for Sigma2D, 2x3 row-major
    double Jp[6];  // dp/dt: J, except for a guarded pinhole direction
    double dirc[2];    // pinhole: t_x / t_z, t_y / t_z after the guard
    bool clamped[2];   // pinhole: whether the guard clamped each
    double M[6];   // J W
    double qn[4], qnorm, Rq[9];
    double S[3];
    double V[6];   // M Rq diag(S)
    double a, b, c, det;  // Sigma2D = [[a, b], [b, c]]
    double dir[3], vnorm; // unit direction camera centre -> m (world frame)
};

// Eq. 1, 3-5, 9-16 (or Eq. 2 for a pinhole camera).  Returns false when the
// Gaussian is culled (inside the near sphere / in front of the near plane,
// opacity that can never pass alpha_min, on the polar axis of the ERP
// camera, or a degenerate 2D covariance).
__device__ inline bool project_core(const ProjectArgs &A, int64_t i, double o, Proj &P) {
    const double m0 = A.means[3 * i], m1 = A.means[3 * i + 1], m2 = A.means[3 * i + 2];
    for (int r = 0; r < 3; ++r) P.t[r] = A.R[3 * r] * m0 + A.R[3 * r + 1] * m1 + A.R[3 * r + 2] * m2 + A.t[r];
    const double tx = P.t[0], ty = P.t[1], tz = P.t[2];
    const double rho2 = tx * tx + tz * tz;
    P.rho = sqrt(rho2);
    P.tr = sqrt(rho2 + ty * ty);
    if (A.model == OMNIGS_CAMERA_PINHOLE) {
        if (!(tz > A.near_plane) || !(o > A.alpha_min)) return false;
        P.depth = tz;
        P.px = A.fx * tx / tz + A.cx;
        P.py = A.fy * ty / tz + A.cy;
        const double ax = tx / tz, ay = ty / tz;
        const double mx = (0.5 * A.width - A.cx) / A.fx, hx = 1.3 * 0.5 * A.width / A.fx;
        const double my = (0.5 * A.height - A.cy) / A.fy, hy = 1.3 * 0.5 * A.height / A.fy;
        P.dirc[0] = ax < mx - hx ? mx - hx : (ax > mx + hx ? mx + hx : ax);
        P.dirc[1] = ay < my - hy ? my - hy : (ay > my + hy ? my + hy : ay);
        P.clamped[0] = P.dirc[0] != ax;
        P.clamped[1] = P.dirc[1] != ay;
        P.J[0] = A.fx / tz;
        P.J[1] = 0.0;
        P.J[2] = -A.fx * P.dirc[0] / tz;
        P.J[3] = 0.0;
        P.J[4] = A.fy / tz;
        P.J[5] = -A.fy * P.dirc[1] / tz;
        for (int k = 0; k < 6; ++k) P.Jp[k] = P.J[k];
        P.Jp[2] = -A.fx * ax / tz;
        P.Jp[5] = -A.fy * ay / tz;
    } else {
        if (!(P.tr > A.near_plane) || !(o > A.alpha_min) || !(P.rho > 1e-6 * P.tr)) return false;
        P.depth = P.tr;
        double lon = atan2(tx, tz);
        if (lon >= kPi) lon = -kPi;
        // one reciprocal per denominator, multiplied in (a double division is
        // a long dependent sequence; the product differs in the last bit)
        const double itr = 1.0 / P.tr;
        const double lat = asin(ty * itr);
        P.px = (lon * kInvPi + 1.0) * (0.5 * A.width);
        P.py = (2.0 * lat * kInvPi + 1.0) * (0.5 * A.height);
        const double kx = A.width * (0.5 * kInvPi), ky = A.height * kInvPi;
        const double irho2 = 1.0 / rho2, ir2 = itr * itr, ir2rho = ir2 / P.rho;
        P.J[0] = kx * tz * irho2;
        P.J[1] = 0.0;
        P.J[2] = -kx * tx * irho2;
        P.J[3] = -ky * tx * ty * ir2rho;
        P.J[4] = ky * P.rho * ir2;
        P.J[5] = -ky * tz * ty * ir2rho;
        for (int k = 0; k < 6; ++k) P.Jp[k] = P.J[k];
    }
    for (int a = 0; a < 2; ++a)
        for (int k = 0; k < 3; ++k)
            P.M[3 * a + k] = P.J[3 * a] * A.R[k] + P.J[3 * a + 1] * A.R[3 + k] + P.J[3 * a + 2] * A.R[6 + k];
    const float4 q = reinterpret_cast<const float4 *>(A.quats)[i];
    P.qnorm = sqrt((double)q.x * q.x + (double)q.y * q.y + (double)q.z * q.z + (double)q.w * q.w);
    if (!(P.qnorm > 0.0)) return false;
    const double iqn = 1.0 / P.qnorm;
    const double w = q.x * iqn, x = q.y * iqn, y = q.z * iqn, z = q.w * iqn;
    P.qn[0] = w; P.qn[1] = x; P.qn[2] = y; P.qn[3] = z;
    double *R = P.Rq;
    R[0] = 1.0 - 2.0 * (y * y + z * z); R[1] = 2.0 * (x * y - w * z);       R[2] = 2.0 * (x * z + w * y);
    R[3] = 2.0 * (x * y + w * z);       R[4] = 1.0 - 2.0 * (x * x + z * z); R[5] = 2.0 * (y * z - w * x);
    R[6] = 2.0 * (x * z - w * y);       R[7] = 2.0 * (y * z + w * x);       R[8] = 1.0 - 2.0 * (x * x + y * y);
    for (int k = 0; k < 3; ++k) P.S[k] = A.scales[3 * i + k];
    for (int a = 0; a < 2; ++a)
        for (int k = 0; k < 3; ++k)
            P.V[3 * a + k] = (P.M[3 * a] * R[k] + P.M[3 * a + 1] * R[3 + k] + P.M[3 * a + 2] * R[6 + k]) * P.S[k];
    const double *V0 = P.V, *V1 = P.V + 3;
    P.a = V0[0] * V0[0] + V0[1] * V0[1] + V0[2] * V0[2] + A.dilation;
    P.b = V0[0] * V1[0] + V0[1] * V1[1] + V0[2] * V1[2];
    P.c = V1[0] * V1[0] + V1[1] * V1[1] + V1[2] * V1[2] + A.dilation;
    P.det = P.a * P.c - P.b * P.b;
    if (!(P.det > 0.0)) return false;
    const double v0 = m0 - A.campos[0], v1 = m1 - A.campos[1], v2 = m2 - A.campos[2];
    P.vnorm = sqrt(v0 * v0 + v1 * v1 + v2 * v2);
    const double ivn = 1.0 / P.vnorm;
    P.dir[0] = v0 * ivn;
    P.dir[1] = v1 * ivn;
    P.dir[2] = v2 * ivn;
    return true;
}

// Projection of Gaussian i for the camera of A; the outputs go to index
// `slot` of the output arrays.
template <int D>
__device__ inline uint32_t project_one(const ProjectArgs &A, int64_t i, int64_t slot, BlendRecord *rec,
                                       uint32_t *depth_key, float *depth, uint32_t *n_tiles, uint2 *rect,
                                       uint32_t *n_super, float *radii) {
    const double o = A.opacities[i];
    Proj P;
    bool vis = project_core(A, i, o, P);
    uint32_t ntx = 0, nty = 0, tx0 = 0, ty0 = 0;
    double radius = 0.0;
    if (vis) {
        const double kcut = 2.0 * log(o / A.alpha_min);
        const double ex = sqrt(kcut * P.a), ey = sqrt(kcut * P.c);
        radius = fmax(ex, ey);
        double xs = ceil(P.px - ex - 0.5), xe = floor(P.px + ex - 0.5);
        double ys = ceil(P.py - ey - 0.5), ye = floor(P.py + ey - 0.5);
        ys = fmax(ys, 0.0);
        ye = fmin(ye, (double)(A.rows - 1));  // the rendered rows
        const bool pinhole = A.model == OMNIGS_CAMERA_PINHOLE;
        if (pinhole) {  // no seam: columns clamp like rows
            xs = fmax(xs, 0.0);
            xe = fmin(xe, (double)(A.width - 1));
        }
        const bool full = !pinhole && (xe - xs + 1.0) >= (double)A.width;
        if ((!full && xe < xs) || ye < ys) {
            vis = false;
        } else {
            if (pinhole) {
                tx0 = (uint32_t)((int)xs / kTile);
                ntx = (uint32_t)((int)xe / kTile) - tx0 + 1;
            } else if (full) {
                tx0 = 0;
                ntx = A.tiles_x;
            } else {
                // xs, xe lie within (-W, 2W): exact in int
                const int t0 = (int)floor(xs / kTile), t1 = (int)floor(xe / kTile);
                const int cnt = t1 - t0 + 1;
                if (cnt >= A.tiles_x) {
                    tx0 = 0;
                    ntx = A.tiles_x;
                } else {
                    tx0 = (uint32_t)(((t0 % A.tiles_x) + A.tiles_x) % A.tiles_x);
                    ntx = (uint32_t)cnt;
                }
            }
            ty0 = (uint32_t)((int)ys / kTile);
            nty = (uint32_t)((int)ye / kTile) - ty0 + 1;
        }
    }
    if (!vis) {
        depth_key[slot] = kCulledKey;
        if (depth) depth[slot] = 0.0f;
        n_tiles[slot] = 0;
        rect[slot] = make_uint2(0, 0);
        n_super[slot] = 0;
        if (radii) radii[slot] = 0.0f;
        return 0u;
    }
    constexpr int K = (D + 1) * (D + 1);
    double Y[16];
    sh_basis<D>(P.dir[0], P.dir[1], P.dir[2], Y);
    // all coefficient loads issued together (kept ahead of their use by a
    // scheduling barrier), held as floats (not doubles)
    float shp[K * 3];
    {
        const float *src = A.sh + i * (int64_t)A.sh_coeffs * 3;
#pragma unroll
        for (int k = 0; k < K * 3; ++k) shp[k] = src[k];
    }
    __builtin_amdgcn_sched_barrier(0);
    double v[3] = {0.5, 0.5, 0.5};
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) v[ch] += Y[k] * (double)shp[3 * k + ch];
    float rgb[3];
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) rgb[ch] = v[ch] < 0.0 ? 0.0f : (float)v[ch];
    BlendRecord r;
    r.px_hi = (float)P.px;
    r.px_lo = (float)(P.px - (double)r.px_hi);
    r.py_hi = (float)P.py;
    r.py_lo = (float)(P.py - (double)r.py_hi);
    // Q = Sigma2D^-1 = L L^T with L = [[l00, 0], [l10, l11]]:
    // l00 = sqrt(c / det), l10 = -b / sqrt(c det), l11 = 1 / sqrt(c); the
    // blend evaluates d^T Q d as |L^T d|^2, a sum of two squares, which keeps
    // its precision for elongated footprints seen from far away (centres
    // thousands of pixels off a pinhole image), where the three terms of the
    // expanded form cancel.  Scaled by sqrt(log2(e) / 2): log2 G = -|L^T d|^2.
    const double ls = sqrt(0.5 * 1.4426950408889634074), sc = sqrt(P.c);
    r.l00 = (float)(ls * sqrt(P.c / P.det));
    r.l10 = (float)(ls * (-P.b / (sc * sqrt(P.det))));
    r.l11 = (float)(ls / sc);
    r.log2o = (float)log2(o);
    r.r = rgb[0];
    r.g = rgb[1];
    r.b = rgb[2];
    r.reach = (float)(log2(o / A.alpha_min));
    float4 *dst = reinterpret_cast<float4 *>(rec + slot);
    dst[0] = make_float4(r.px_hi, r.px_lo, r.py_hi, r.py_lo);
    dst[1] = make_float4(r.l00, r.l10, r.l11, r.log2o);
    dst[2] = make_float4(r.r, r.g, r.b, r.reach);
    depth_key[slot] = __float_as_uint((float)P.depth);
    if (depth) depth[slot] = (float)P.depth;
    n_tiles[slot] = ntx * nty;
    const uint2 tr = make_uint2(tx0 | (ntx << 16), ty0 | (nty << 16));
    rect[slot] = tr;
    const uint2 sr = super_rect(tr, A.tiles_x);
    n_super[slot] = (sr.x >> 16) * (sr.y >> 16);
    if (radii) radii[slot] = (float)radius;
    return ntx * nty;
}

// Adds the sum of v over the 256-thread block to *total (one atomic per
// block; integer, so the result does not depend on the order).
__device__ inline void add_block_total(uint32_t v, uint32_t *total) {
    __shared__ uint32_t part[4];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    if (__lane_id() == 0) part[threadIdx.x / kWave] = v;
    __syncthreads();
    if (threadIdx.x == 0) atomicAdd(total, part[0] + part[1] + part[2] + part[3]);
}

template <int D>
__global__ __launch_bounds__(256) void k_project(ProjectArgs A, BlendRecord *rec, uint32_t *depth_key, float *depth,
                                                 uint32_t *n_tiles, uint2 *rect, uint32_t *n_super, float *radii,
                                                 uint32_t *tiles_total) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t covered = 0;
    if (i < A.n) covered = project_one<D>(A, i, i, rec, depth_key, depth, n_tiles, rect, n_super, radii);
    add_block_total(covered, tiles_total);
}

// Every camera of a batch for Gaussian i in turn: the Gaussian's parameters
// are fetched from HBM once and re-read from cache for the later cameras.
template <int D>
__global__ __launch_bounds__(256) void k_project_batch(ProjectArgs A, CamTable T, BlendRecord *rec,
                                                       uint32_t *depth_key, float *depth, uint32_t *n_tiles,
                                                       uint2 *rect, uint32_t *n_super, uint32_t *tiles_total) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t covered = 0;
    for (int b = 0; b < T.count && i < A.n; ++b) {
        ProjectArgs C = A;
        const CamGeom &g = T.c[b];
        for (int k = 0; k < 9; ++k) C.R[k] = g.R[k];
        for (int k = 0; k < 3; ++k) {
            C.t[k] = g.t[k];
            C.campos[k] = g.campos[k];
        }
        C.width = g.width;
        C.height = g.height;
        C.tiles_x = g.tiles_x;
        C.tiles_y = g.tiles_y;
        C.rows = g.rows;
        C.model = g.model;
        C.fx = g.fx;
        C.fy = g.fy;
        C.cx = g.cx;
        C.cy = g.cy;
        covered += project_one<D>(C, i, (int64_t)b * A.n + i, rec, depth_key, depth, n_tiles, rect, n_super,
                                  nullptr);
    }
    add_block_total(covered, tiles_total);
}

// dJ/dt for the pinhole Jacobian J00 = fx / tz, J02 = -fx a / tz,
// J11 = fy / tz, J12 = -fy b / tz (a = t_x / t_z, b = t_y / t_z, each
// constant in t where the guard clamped it): dJ[e][n] = d J_e / d t_n.
__device__ inline void jacobian_grad_pinhole(const Proj &P, double fx, double fy, double (*dJ)[3]) {
    const double tz = P.t[2], iz2 = 1.0 / (tz * tz), iz3 = iz2 / tz;
    for (int e = 0; e < 6; ++e) dJ[e][0] = dJ[e][1] = dJ[e][2] = 0.0;
    dJ[0][2] = -fx * iz2;
    dJ[4][2] = -fy * iz2;
    if (P.clamped[0]) {
        dJ[2][2] = fx * P.dirc[0] * iz2;
    } else {
        dJ[2][0] = -fx * iz2;
        dJ[2][2] = 2.0 * fx * P.t[0] * iz3;
    }
    if (P.clamped[1]) {
        dJ[5][2] = fy * P.dirc[1] * iz2;
    } else {
        dJ[5][1] = -fy * iz2;
        dJ[5][2] = 2.0 * fy * P.t[1] * iz3;
    }
}

// dJ/dt for the spherical Jacobian: dJ[e][n] = d J_e / d t_n, e = 3a + j.
__device__ inline void jacobian_grad(const Proj &P, double kx, double ky, double (*dJ)[3]) {
    const double tx = P.t[0], ty = P.t[1], tz = P.t[2];
    const double rho = P.rho, rho2 = rho * rho, rho4 = rho2 * rho2;
    const double r2 = P.tr * P.tr, r4 = r2 * r2;
    const double rho3 = rho2 * rho;
    const double txx_tzz = tx * tx - tz * tz;
    // the denominators' reciprocals, multiplied in
    const double irho4 = 1.0 / rho4, ir4 = 1.0 / r4, ir4rho = ir4 / rho, ir4rho3 = ir4rho / rho2;
    dJ[0][0] = -2.0 * kx * tx * tz * irho4;
    dJ[0][1] = 0.0;
    dJ[0][2] = kx * txx_tzz * irho4;
    dJ[1][0] = dJ[1][1] = dJ[1][2] = 0.0;
    dJ[2][0] = kx * txx_tzz * irho4;
    dJ[2][1] = 0.0;
    dJ[2][2] = 2.0 * kx * tx * tz * irho4;
    const double q = 2.0 * rho2 + r2;
    const double u = ty * ty - rho2;
    dJ[3][0] = -ky * ty * (r2 * rho2 - tx * tx * q) * ir4rho3;
    dJ[3][1] = ky * tx * u * ir4rho;
    dJ[3][2] = ky * tx * ty * tz * q * ir4rho3;
    dJ[4][0] = ky * tx * u * ir4rho;
    dJ[4][1] = -2.0 * ky * rho * ty * ir4;
    dJ[4][2] = ky * tz * u * ir4rho;
    dJ[5][0] = ky * tx * ty * tz * q * ir4rho3;
    dJ[5][1] = ky * tz * u * ir4rho;
    dJ[5][2] = -ky * ty * (r2 * rho2 - tz * tz * q) * ir4rho3;
}

template <int D>
__global__ __launch_bounds__(256) void k_project_backward(ProjectArgs A, const uint32_t *n_tiles, const float *acc,
                                                          int acc_stride, omnigs_grads G) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= A.n) return;
    const int K = A.sh_coeffs;
    float *dsh = G.dsh + i * (int64_t)K * 3;
    constexpr int KD = (D + 1) * (D + 1);
    for (int k = KD; k < K; ++k) dsh[3 * k] = dsh[3 * k + 1] = dsh[3 * k + 2] = 0.0f;
    const double o = A.opacities[i];
    Proj P;
    if (n_tiles[i] == 0 || !project_core(A, i, o, P)) {
        for (int k = 0; k < 3; ++k) G.dmeans[3 * i + k] = G.dscales[3 * i + k] = 0.0f;
        reinterpret_cast<float4 *>(G.dquats)[i] = make_float4(0.f, 0.f, 0.f, 0.f);
        G.dopacities[i] = 0.0f;
        for (int k = 0; k < KD; ++k) dsh[3 * k] = dsh[3 * k + 1] = dsh[3 * k + 2] = 0.0f;
        G.dscreen[2 * i] = G.dscreen[2 * i + 1] = 0.0f;
        return;
    }
    double g[kAccAux];
#pragma unroll
    for (int k = 0; k < kAcc; ++k) g[k] = acc[i * acc_stride + k];
    g[kAcc] = acc_stride > kAcc ? acc[i * acc_stride + kAcc] : 0.0;  // dL/dd of the depth image
    // dL/dSigma2D from the blend's moments M = sum(w w^T gp) of w = Ls^T d,
    // Ls = sqrt(log2(e) / 2) L and Q = Sigma2D^-1 = L L^T: the exponent's
    // gradient 1/2 Q d d^T Q summed with weights gp is
    // 1/2 (2 ln2)^2 Ls M Ls^T = ln2 L M L^T, with
    // L = [[sqrt(c / det), 0], [-b / sqrt(c det), 1 / sqrt(c)]]
    const double sc = sqrt(P.c), sd = sqrt(P.det);
    const double isc = 1.0 / sc, isd = 1.0 / sd;
    const double L0 = sc * isd, L1 = -P.b * (isc * isd), L2 = isc;
    const double m00 = g[2], m01 = g[3], m11 = g[4];
    const double r1 = L1 * m00 + L2 * m01;  // row 1 of L M, first column
    const double S00 = kLn2d * (L0 * L0 * m00);
    const double S01 = kLn2d * (L0 * r1);
    const double S11 = kLn2d * (L1 * r1 + L2 * (L1 * m01 + L2 * m11));
    // a = V0.V0, b = V0.V1, c = V1.V1 (b used twice in the symmetric matrix)
    const double ga = S00, gb = 2.0 * S01, gc = S11;
    double dV[6];
    for (int k = 0; k < 3; ++k) {
        dV[k] = 2.0 * ga * P.V[k] + gb * P.V[3 + k];
        dV[3 + k] = gb * P.V[k] + 2.0 * gc * P.V[3 + k];
    }
    // V = M B, B = Rq diag(S)
    double dM[6], dB[9];
    for (int a = 0; a < 2; ++a)
        for (int j = 0; j < 3; ++j) {
            double v = 0.0;
            for (int k = 0; k < 3; ++k) v += dV[3 * a + k] * P.Rq[3 * j + k] * P.S[k];
            dM[3 * a + j] = v;
        }
    for (int j = 0; j < 3; ++j)
        for (int k = 0; k < 3; ++k) dB[3 * j + k] = P.M[j] * dV[k] + P.M[3 + j] * dV[3 + k];
    double dS[3], dR[9];
    for (int k = 0; k < 3; ++k) {
        dS[k] = dB[k] * P.Rq[k] + dB[3 + k] * P.Rq[3 + k] + dB[6 + k] * P.Rq[6 + k];
        for (int j = 0; j < 3; ++j) dR[3 * j + k] = dB[3 * j + k] * P.S[k];
    }
    // R(q) for the unit quaternion (w, x, y, z)
    const double w = P.qn[0], x = P.qn[1], y = P.qn[2], z = P.qn[3];
    double dqn[4];
    dqn[0] = 2.0 * (-z * dR[1] + y * dR[2] + z * dR[3] - x * dR[5] - y * dR[6] + x * dR[7]);
    dqn[1] = 2.0 * (y * dR[1] + z * dR[2] + y * dR[3] - 2.0 * x * dR[4] - w * dR[5] + z * dR[6] + w * dR[7] -
                    2.0 * x * dR[8]);
    dqn[2] = 2.0 * (-2.0 * y * dR[0] + x * dR[1] + w * dR[2] + x * dR[3] + z * dR[5] - w * dR[6] + z * dR[7] -
                    2.0 * y * dR[8]);
    dqn[3] = 2.0 * (-2.0 * z * dR[0] - w * dR[1] + x * dR[2] + w * dR[3] - 2.0 * z * dR[4] + y * dR[5] +
                    x * dR[6] + y * dR[7]);
    const double qd = w * dqn[0] + x * dqn[1] + y * dqn[2] + z * dqn[3];
    float4 dq;
    const double iqn = 1.0 / P.qnorm;
    dq.x = (float)((dqn[0] - w * qd) * iqn);
    dq.y = (float)((dqn[1] - x * qd) * iqn);
    dq.z = (float)((dqn[2] - y * qd) * iqn);
    dq.w = (float)((dqn[3] - z * qd) * iqn);
    // M = J W: dJ = dM W^T
    double dJ[6];
    for (int a = 0; a < 2; ++a)
        for (int j = 0; j < 3; ++j)
            dJ[3 * a + j] = dM[3 * a] * A.R[3 * j] + dM[3 * a + 1] * A.R[3 * j + 1] + dM[3 * a + 2] * A.R[3 * j + 2];
    double dJdt[6][3];
    if (A.model == OMNIGS_CAMERA_PINHOLE)
        jacobian_grad_pinhole(P, A.fx, A.fy, dJdt);
    else
        jacobian_grad(P, A.width * (0.5 * kInvPi), A.height * kInvPi, dJdt);
    double dt[3];
    const double itr = 1.0 / P.tr;
    for (int nn = 0; nn < 3; ++nn) {
        double v = P.Jp[nn] * g[0] + P.Jp[3 + nn] * g[1];
        for (int e = 0; e < 6; ++e) v += dJ[e] * dJdt[e][nn];
        // the depth value d: t_r (d t_r / dt = t / t_r) or t_z
        v += A.model == OMNIGS_CAMERA_PINHOLE ? (nn == 2 ? g[kAcc] : 0.0) : g[kAcc] * P.t[nn] * itr;
        dt[nn] = v;
    }
    double dm[3];
    for (int k = 0; k < 3; ++k) dm[k] = A.R[k] * dt[0] + A.R[3 + k] * dt[1] + A.R[6 + k] * dt[2];
    // the geometric gradients out before the SH term, so that their values
    // are not held through it
    for (int k = 0; k < 3; ++k) G.dscales[3 * i + k] = (float)dS[k];
    reinterpret_cast<float4 *>(G.dquats)[i] = dq;
    G.dopacities[i] = (float)g[5];
    G.dscreen[2 * i] = (float)(g[0] * (0.5 * A.width));
    G.dscreen[2 * i + 1] = (float)(g[1] * (0.5 * A.height));
    // SH colour: the coefficients loaded once as floats (all loads ahead of
    // the dsh stores, which may alias them), the basis gradient accumulated
    // term by term
    double Y[16];
    sh_basis<D>(P.dir[0], P.dir[1], P.dir[2], Y);
    float shp[KD * 3];
    {
        const float *src = A.sh + i * (int64_t)K * 3;
#pragma unroll
        for (int k = 0; k < KD * 3; ++k) shp[k] = src[k];
    }
    double grgb[3];
    {
        double v[3] = {0.5, 0.5, 0.5};
#pragma unroll
        for (int k = 0; k < KD; ++k)
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) v[ch] += Y[k] * (double)shp[3 * k + ch];
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) grgb[ch] = v[ch] < 0.0 ? 0.0 : g[6 + ch];
    }
    double gdir[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int k = 0; k < KD; ++k) {
        const double s = (double)shp[3 * k] * grgb[0] + (double)shp[3 * k + 1] * grgb[1] +
                         (double)shp[3 * k + 2] * grgb[2];
        double d[3];
        sh_basis_grad_k(k, P.dir[0], P.dir[1], P.dir[2], d);
        gdir[0] += s * d[0];
        gdir[1] += s * d[1];
        gdir[2] += s * d[2];
        dsh[3 * k] = (float)(Y[k] * grgb[0]);
        dsh[3 * k + 1] = (float)(Y[k] * grgb[1]);
        dsh[3 * k + 2] = (float)(Y[k] * grgb[2]);
    }
    const double pd = P.dir[0] * gdir[0] + P.dir[1] * gdir[1] + P.dir[2] * gdir[2];
    const double ivn = 1.0 / P.vnorm;
    for (int k = 0; k < 3; ++k) dm[k] += (gdir[k] - P.dir[k] * pd) * ivn;
    for (int k = 0; k < 3; ++k) G.dmeans[3 * i + k] = (float)dm[k];
}

}  // namespace

hipError_t launch_project(const ProjectArgs &a, BlendRecord *rec, uint32_t *depth_key, float *depth, uint32_t *n_tiles,
                          uint2 *rect, uint32_t *n_super, float *radii, uint32_t *tiles_total, hipStream_t st,
                          bool cleared) {
    hipError_t e = cleared ? hipSuccess : launch_fill_u32(tiles_total, 0u, 1, st);
    if (e != hipSuccess || a.n == 0) return e;
    const dim3 grid((unsigned)((a.n + 255) / 256));
    switch (a.sh_degree) {
        case 0: hipLaunchKernelGGL(k_project<0>, grid, dim3(256), 0, st, a, rec, depth_key, depth, n_tiles, rect, n_super, radii, tiles_total); break;
        case 1: hipLaunchKernelGGL(k_project<1>, grid, dim3(256), 0, st, a, rec, depth_key, depth, n_tiles, rect, n_super, radii, tiles_total); break;
        case 2: hipLaunchKernelGGL(k_project<2>, grid, dim3(256), 0, st, a, rec, depth_key, depth, n_tiles, rect, n_super, radii, tiles_total); break;
        default: hipLaunchKernelGGL(k_project<3>, grid, dim3(256), 0, st, a, rec, depth_key, depth, n_tiles, rect, n_super, radii, tiles_total); break;
    }
    return hipGetLastError();
}

hipError_t launch_project_batch(const ProjectArgs &a, const CamTable &cams, BlendRecord *rec, uint32_t *depth_key,
                                float *depth, uint32_t *n_tiles, uint2 *rect, uint32_t *n_super,
                                uint32_t *tiles_total, hipStream_t st) {
    hipError_t e = launch_fill_u32(tiles_total, 0u, 1, st);
    if (e != hipSuccess || a.n == 0 || cams.count == 0) return e;
    const dim3 grid((unsigned)((a.n + 255) / 256));
    switch (a.sh_degree) {
        case 0: hipLaunchKernelGGL(k_project_batch<0>, grid, dim3(256), 0, st, a, cams, rec, depth_key, depth, n_tiles, rect, n_super, tiles_total); break;
        case 1: hipLaunchKernelGGL(k_project_batch<1>, grid, dim3(256), 0, st, a, cams, rec, depth_key, depth, n_tiles, rect, n_super, tiles_total); break;
        case 2: hipLaunchKernelGGL(k_project_batch<2>, grid, dim3(256), 0, st, a, cams, rec, depth_key, depth, n_tiles, rect, n_super, tiles_total); break;
        default: hipLaunchKernelGGL(k_project_batch<3>, grid, dim3(256), 0, st, a, cams, rec, depth_key, depth, n_tiles, rect, n_super, tiles_total); break;
    }
    return hipGetLastError();
}

hipError_t launch_project_backward(const ProjectArgs &a, const uint32_t *n_tiles, const float *acc, int acc_stride,
                                   const omnigs_grads &gr, hipStream_t st) {
    if (a.n == 0) return hipSuccess;
    const dim3 grid((unsigned)((a.n + 255) / 256));
    switch (a.sh_degree) {
        case 0: hipLaunchKernelGGL(k_project_backward<0>, grid, dim3(256), 0, st, a, n_tiles, acc, acc_stride, gr); break;
        case 1: hipLaunchKernelGGL(k_project_backward<1>, grid, dim3(256), 0, st, a, n_tiles, acc, acc_stride, gr); break;
        case 2: hipLaunchKernelGGL(k_project_backward<2>, grid, dim3(256), 0, st, a, n_tiles, acc, acc_stride, gr); break;
        default: hipLaunchKernelGGL(k_project_backward<3>, grid, dim3(256), 0, st, a, n_tiles, acc, acc_stride, gr); break;
    }
    return hipGetLastError();
}

}  // namespace omnigs
