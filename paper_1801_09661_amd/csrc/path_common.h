// Device helpers shared by the path kernels: the thresholding operators of
// Section 2.2, penalty values and derivatives, wave reductions.
#pragma once

#include "oem_internal.h"

namespace oem {

constexpr int kPathThreads = 256;
constexpr int kPathWaves = kPathThreads / kWave;

// ---------------------------------------------------------------- updates

__device__ inline double sgn(double v) { return v > 0.0 ? 1.0 : (v < 0.0 ? -1.0 : 0.0); }
__device__ inline double pos(double v) { return v > 0.0 ? v : 0.0; }

// Scalar thresholding operators of Section 2.2 (lam_w = w_j * lambda).
__device__ inline double update1(int kind, double u, double lam_w, double d, double alpha,
                                 double gamma)
{
    const double au = fabs(u);
    switch (kind) {
    case OEM_LASSO:  // S(u, w lambda, d)
        return sgn(u) * pos(au - lam_w) / d;
    case OEM_ENET:
        return sgn(u) * pos(au - lam_w * alpha) / (d + lam_w * (1.0 - alpha));
    case OEM_MCP:    // M(u, w lambda, gamma, d)
        if (au <= lam_w * gamma * d) return sgn(u) * gamma * pos(au - lam_w) / (gamma * d - 1.0);
        return u / d;
    case OEM_SCAD:   // C(u, w lambda, gamma, d)
        if (au <= (d + 1.0) * lam_w) return sgn(u) * pos(au - lam_w) / d;
        if (au <= lam_w * gamma * d)
            return sgn(u) * ((gamma - 1.0) * au - lam_w * gamma) / ((gamma - 1.0) * d - 1.0);
        return u / d;
    default:
        return 0.0;
    }
}

// The same updates with the divisors of Section 2.2 replaced by reciprocals
// fixed for one (coordinate, lambda): the iteration then needs no division.
struct Upd {
    double thr;    // soft-threshold level: w lambda (w lambda alpha for the elastic net)
    double s1;     // scale of the soft-thresholded value
    double t1;     // SCAD: end of the soft region, (d + 1) w lambda
    double t2;     // MCP / SCAD: start of the unpenalised region, w lambda gamma d
    double c2;     // SCAD: w lambda gamma
    double s2;     // SCAD: 1 / ((gamma - 1) d - 1)
    double inv_d;  // 1 / d
};

__device__ inline Upd make_upd(int kind, double lam_w, double d, double alpha, double gamma)
{
    Upd q;
    q.inv_d = 1.0 / d;
    q.thr = lam_w;
    q.s1 = q.inv_d;
    q.t1 = q.t2 = INFINITY;
    q.c2 = 0.0;
    q.s2 = 0.0;
    if (kind == OEM_ENET) {
        q.thr = lam_w * alpha;
        q.s1 = 1.0 / (d + lam_w * (1.0 - alpha));
    } else if (kind == OEM_MCP) {
        q.s1 = gamma / (gamma * d - 1.0);
        q.t1 = q.t2 = lam_w * gamma * d;
    } else if (kind == OEM_SCAD) {
        q.t1 = (d + 1.0) * lam_w;
        q.t2 = lam_w * gamma * d;
        q.c2 = lam_w * gamma;
        q.s2 = 1.0 / ((gamma - 1.0) * d - 1.0);
    }
    return q;
}

// MCP and SCAD share the form: soft region up to t1, a linear middle piece
// up to t2 (SCAD only; empty for MCP since t1 = t2), u / d beyond.
__device__ inline double update_fast(int kind, double u, const Upd &q, double gamma)
{
    const double au = fabs(u);
    const double soft = copysign(pos(au - q.thr) * q.s1, u);
    if (kind == OEM_LASSO || kind == OEM_ENET) return soft;
    if (au <= q.t1) return soft;
    if (au <= q.t2) return copysign(((gamma - 1.0) * au - q.c2) * q.s2, u);
    return u * q.inv_d;
}

// derivative of the penalty at |b| > 0 (for the stationarity check)
__device__ inline double pen_deriv(int kind, double ab, double lw, double alpha, double gamma)
{
    switch (kind) {
    case OEM_LASSO: return lw;
    case OEM_ENET: return alpha * lw + (1.0 - alpha) * lw * ab;
    case OEM_MCP: return pos(lw - ab / gamma);
    case OEM_SCAD:
        if (ab <= lw) return lw;
        if (ab <= gamma * lw) return (gamma * lw - ab) / (gamma - 1.0);
        return 0.0;
    default: return 0.0;
    }
}

__device__ inline double pen_value(int kind, double b, double lw, double alpha, double gamma)
{
    const double ab = fabs(b);
    switch (kind) {
    case OEM_LASSO: return lw * ab;
    case OEM_ENET: return alpha * lw * ab + 0.5 * (1.0 - alpha) * lw * b * b;
    case OEM_MCP: return ab <= gamma * lw ? lw * ab - b * b / (2.0 * gamma) : 0.5 * gamma * lw * lw;
    case OEM_SCAD:
        if (ab <= lw) return lw * ab;
        if (ab <= gamma * lw) return -(ab * ab - 2.0 * gamma * lw * ab + lw * lw) / (2.0 * (gamma - 1.0));
        return 0.5 * (gamma + 1.0) * lw * lw;
    default: return 0.0;
    }
}

// ---------------------------------------------------------------- group penalties

// Update of one group from nrm = ||u_g|| (for the sparse group lasso:
// ||v_g||, v = the soft-thresholded u): beta_j = group_update_one(u_j).
// eq. glasso: (u/d)(1 - c lambda / ||u||)_+; eqs. gmcp, gscad: the scalar
// MCP / SCAD update of ||u|| at c lambda along u / ||u||.
struct GroupUpd {
    int kind;       // OEM_GRP_LASSO (also the outer step of OEM_SGL) or OEM_GRP_MCP / SCAD
    double f;       // group lasso factor 1 - lam_c / nrm (zero group when <= 0)
    double t;       // MCP / SCAD: updated norm (zero group when <= 0)
    double nrm;
    double d;
};

__device__ inline GroupUpd make_group_upd(int kind, double nrm, double lam_c, double d, double gamma)
{
    GroupUpd g;
    g.kind = (kind == OEM_SGL) ? OEM_GRP_LASSO : kind;
    g.nrm = nrm;
    g.d = d;
    g.f = nrm > 0.0 ? 1.0 - lam_c / nrm : 0.0;
    g.t = 0.0;
    if (kind == OEM_GRP_MCP || kind == OEM_GRP_SCAD)
        g.t = nrm > 0.0 ? update1(kind == OEM_GRP_MCP ? OEM_MCP : OEM_SCAD, nrm, lam_c, d, 0.0, gamma) : 0.0;
    return g;
}

__device__ inline double group_update_one(const GroupUpd &g, double u)
{
    if (g.kind == OEM_GRP_LASSO) return g.f > 0.0 ? (u / g.d) * g.f : 0.0;
    return g.t > 0.0 ? g.t * (u / g.nrm) : 0.0;
}

// the group's threshold level: c lambda, or c lambda (1 - tau) for the outer
// step of the sparse group lasso
__device__ inline double group_lam_c(int kind, double cgk, double lam, double tau)
{
    return kind == OEM_SGL ? cgk * lam * (1.0 - tau) : cgk * lam;
}

// inner soft threshold of the sparse group lasso (no division by d)
__device__ inline double sgl_inner(double u, double w, double lam, double tau)
{
    return sgn(u) * pos(fabs(u) - w * lam * tau);
}

// penalty of one group: bn = ||beta_g||, l1w = sum_j w_j |beta_j|
__device__ inline double group_pen_value(int kind, double bn, double l1w, double cgk, double lam,
                                         double gamma, double tau)
{
    const double lc = lam * cgk;
    switch (kind) {
    case OEM_GRP_MCP: return pen_value(OEM_MCP, bn, lc, 0.0, gamma);
    case OEM_GRP_SCAD: return pen_value(OEM_SCAD, bn, lc, 0.0, gamma);
    case OEM_SGL: return (1.0 - tau) * lc * bn + tau * lam * l1w;
    default: return lc * bn;
    }
}

// derivative of a radial group penalty at ||beta_g|| = bn > 0
__device__ inline double group_pen_deriv(int kind, double bn, double lc, double gamma)
{
    if (kind == OEM_GRP_MCP) return pen_deriv(OEM_MCP, bn, lc, 0.0, gamma);
    if (kind == OEM_GRP_SCAD) return pen_deriv(OEM_SCAD, bn, lc, 0.0, gamma);
    return lc;
}

// ---------------------------------------------------------------- reductions

// Cross-lane moves with DPP (a 64-bit value moves as two 32-bit halves).
template <int CTRL> __device__ inline double dpp_mov(double v)
{
    int lo = __double2loint(v), hi = __double2hiint(v);
    lo = __builtin_amdgcn_update_dpp(0, lo, CTRL, 0xF, 0xF, false);
    hi = __builtin_amdgcn_update_dpp(0, hi, CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}

__device__ inline double readlane_d(double v, int l)
{
    int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
    int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
    return __hiloint2double(hi, lo);
}

// Wave-wide max / sum: butterfly inside each 16-lane row (quad_perm xor 1,
// xor 2, row rotate 4, 8), then the four row results read out lane by lane.
// The result is the same value in every lane.
__device__ inline double wave_max(double v)
{
    v = fmax(v, dpp_mov<0xB1>(v));
    v = fmax(v, dpp_mov<0x4E>(v));
    v = fmax(v, dpp_mov<0x124>(v));
    v = fmax(v, dpp_mov<0x128>(v));
    return fmax(fmax(readlane_d(v, 0), readlane_d(v, 16)), fmax(readlane_d(v, 32), readlane_d(v, 48)));
}

__device__ inline double wave_sum(double v)
{
    v = v + dpp_mov<0xB1>(v);
    v = v + dpp_mov<0x4E>(v);
    v = v + dpp_mov<0x124>(v);
    v = v + dpp_mov<0x128>(v);
    return (readlane_d(v, 0) + readlane_d(v, 16)) + (readlane_d(v, 32) + readlane_d(v, 48));
}

// max for values that are not NaN (no quieting of signalling NaNs needed)
__device__ inline double nmax(double a, double b) { return a > b ? a : b; }

template <int CTRL> __device__ inline double dpp_get(double v)
{
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, true);
    return __hiloint2double(hi, lo);
}

// Max over lanes 0 .. N-1, valid in lane 0; the other lanes of those rows
// must hold values not above the max (e.g. zero).  Butterfly inside each
// 16-lane row: quad_perm xor 1, xor 2, half-row mirror, row mirror; the rows
// are then joined through lanes 16, 32 and 48.
template <int N> __device__ inline double lanes_max(double v)
{
    if (N > 1) v = nmax(v, dpp_get<0xB1>(v));
    if (N > 2) v = nmax(v, dpp_get<0x4E>(v));
    if (N > 4) v = nmax(v, dpp_get<0x141>(v));
    if (N > 8) v = nmax(v, dpp_get<0x140>(v));
    if (N > 16) v = nmax(v, readlane_d(v, 16));
    if (N > 32) v = nmax(v, nmax(readlane_d(v, 32), readlane_d(v, 48)));
    return v;
}

} // namespace oem
