// geometry.cpp -- host-side reduction of the cone-beam geometry to the ray
// tables of kct_internal.h.  Everything is computed in double precision and
// rounded once to single precision.
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "kct_internal.h"

namespace kct {

void set_error(const std::string &msg);

static bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

// Returns "" when the description is usable, else the reason.
std::string validate_geometry(const kct_volume_desc &v, const kct_cone_desc &c)
{
    if (v.nx <= 0 || v.ny <= 0 || v.nz <= 0) return "volume counts must be positive";
    if ((int64_t)v.nx * v.ny * v.nz >= (int64_t)1 << 31) return "volume has 2^31 voxels or more";
    if (v.nx > (1 << 20) || v.ny > (1 << 20) || v.nz > (1 << 20)) return "volume side above 2^20 voxels";
    if (!finite_pos(v.vx) || !finite_pos(v.vy) || !finite_pos(v.vz)) return "voxel sizes must be positive";
    if (!std::isfinite(v.cx) || !std::isfinite(v.cy) || !std::isfinite(v.cz)) return "volume centre not finite";
    if (c.n_views <= 0 || c.nu <= 0 || c.nv <= 0) return "view and detector counts must be positive";
    if ((int64_t)c.n_views * c.nu * c.nv >= (int64_t)1 << 31) return "projection data has 2^31 rays or more";
    // the backprojector addresses one view's projection values by 32-bit byte offsets
    if ((int64_t)c.nu * c.nv >= (int64_t)1 << 28) return "detector has 2^28 pixels or more";
    if (!finite_pos(c.du) || !finite_pos(c.dv)) return "pixel pitch must be positive";
    if (!finite_pos(c.sid) || !finite_pos(c.sdd)) return "SID and SDD must be positive";
    if (!(c.sdd > c.sid)) return "SDD must exceed SID";
    if (!std::isfinite(c.off_u) || !std::isfinite(c.off_v)) return "detector offset not finite";
    if (!c.angles && (!std::isfinite(c.angle0) || !std::isfinite(c.arc))) return "angle0/arc not finite";
    return "";
}

// Offset h of an axis' index frame (plane m at m - h): the multiple of 1/2 in
// [0, n] nearest to the index of coordinate 0, where the lower corner is at lo
// and cells are v wide.  Exactly n/2 when the axis is centred on 0.
static double plane_offset(double lo, double v, int n)
{
    double h = std::round(-2.0 * lo / v) * 0.5;
    return h < 0.0 ? 0.0 : (h > (double)n ? (double)n : h);
}

static double view_angle(const kct_cone_desc &c, int k)
{
    if (c.angles) return c.angles[k];
    return c.angle0 + (double)k * (c.arc / (double)c.n_views);
}

// Ray tables and kernel constants of a validated description (host memory).
kct_status geometry_tables(const kct_volume_desc &vol, const kct_cone_desc &cone, std::vector<ColParam> &cols,
                           std::vector<RowParam> &rows, std::vector<ViewParam> &views, GeoDev &d)
{
    std::string why = validate_geometry(vol, cone);
    if (!why.empty()) {
        set_error("kct_geometry_create: " + why);
        return KCT_ERR_INVALID_ARG;
    }
    if (cone.angles)
        for (int k = 0; k < cone.n_views; ++k)
            if (!std::isfinite(cone.angles[k])) {
                set_error("kct_geometry_create: view angle not finite");
                return KCT_ERR_INVALID_ARG;
            }
    const int nu = cone.nu, nv = cone.nv, nk = cone.n_views;
    cols.assign((size_t)nk * nu, ColParam{});
    rows.assign(nv, RowParam{});
    views.assign(nk, ViewParam{});

    const double X0 = vol.cx - 0.5 * vol.nx * vol.vx, Y0 = vol.cy - 0.5 * vol.ny * vol.vy;
    const double Z0 = vol.cz - 0.5 * vol.nz * vol.vz;
    const double X1 = X0 + vol.nx * vol.vx, Y1 = Y0 + vol.ny * vol.vy, Z1 = Z0 + vol.nz * vol.vz;
    // Index frame of each axis: plane m sits at m - h, h the multiple of 1/2 in
    // [0, n] nearest to the isocentre's index (n/2 for a centred volume).  A
    // ray nearly parallel to an axis' planes has a crossing that moves by
    // (coordinate error) / slope; such rays pass near the isocentre, where
    // coordinates measured from it are small and carry small rounding errors.
    const double hx = plane_offset(X0, vol.vx, vol.nx), hy = plane_offset(Y0, vol.vy, vol.ny);
    const double hz = plane_offset(Z0, vol.vz, vol.nz);
    // world coordinates of each frame's origin (the volume centre when centred)
    const double ox = vol.cx + (hx - 0.5 * vol.nx) * vol.vx, oy = vol.cy + (hy - 0.5 * vol.ny) * vol.vy;
    const double oz = vol.cz + (hz - 0.5 * vol.nz) * vol.vz;

    for (int iv = 0; iv < nv; ++iv) {
        double qz = ((double)iv - 0.5 * (nv - 1)) * cone.dv + cone.off_v;
        rows[iv].qz = (float)qz;
        rows[iv].inv_qz = qz != 0.0 ? (float)(1.0 / qz) : 0.0f;
    }

    for (int k = 0; k < nk; ++k) {
        const double t = view_angle(cone, k);
        const double c = std::cos(t), s = std::sin(t);
        const double Sx = cone.sid * c, Sy = cone.sid * s;
        const double Cx = Sx - cone.sdd * c, Cy = Sy - cone.sdd * s;
        // The volume must lie strictly between source and detector: the depth
        // of every corner along the central ray is inside (0, SDD).
        for (int cc = 0; cc < 8; ++cc) {
            double px = (cc & 1) ? X1 : X0, py = (cc & 2) ? Y1 : Y0;
            double depth = (px - Sx) * (-c) + (py - Sy) * (-s);
            if (!(depth > 0.0 && depth < cone.sdd)) {
                set_error("kct_geometry_create: the volume is not strictly between source and detector in view " +
                          std::to_string(k));
                return KCT_ERR_INVALID_ARG;
            }
        }
        (void)Z0;
        (void)Z1;
        const int dom = (std::fabs(c) / vol.vx >= std::fabs(s) / vol.vy) ? 0 : 1;
        ViewParam &vp = views[k];
        vp.sx = (float)Sx;
        vp.sy = (float)Sy;
        vp.c = (float)c;
        vp.s = (float)s;
        vp.dom = dom;
        vp.dn = (float)(0.5 * (vol.vx * std::fabs(s) + vol.vy * std::fabs(c)));
        vp.dd = (float)(0.5 * (vol.vx * std::fabs(c) + vol.vy * std::fabs(s)));
        vp.pad = 0;
        const double vxi = dom == 0 ? vol.vx : vol.vy, veta = dom == 0 ? vol.vy : vol.vx;
        const double cxi = dom == 0 ? ox : oy, ceta = dom == 0 ? oy : ox;
        const double Sxi = dom == 0 ? Sx : Sy, Seta = dom == 0 ? Sy : Sx;
        for (int iu = 0; iu < nu; ++iu) {
            const double u = ((double)iu - 0.5 * (nu - 1)) * cone.du + cone.off_u;
            const double Qx = Cx + u * (-s), Qy = Cy + u * c;
            const double Dxi = (dom == 0 ? Qx : Qy) - Sxi;
            const double Deta = (dom == 0 ? Qy : Qx) - Seta;
            const double slope = Deta / Dxi;  // world d eta / d xi
            if (!std::isfinite(slope) || std::fabs(slope) > 8.0) {
                set_error("kct_geometry_create: fan angle too wide (ray more than 82 degrees off the dominant axis)");
                return KCT_ERR_UNSUPPORTED;
            }
            const double t_c = (cxi - Sxi) / Dxi;
            const double eta_w = Seta + Deta * t_c;
            const double a = slope * (vxi / veta);
            const double gp = vxi / Dxi;
            ColParam &cp = cols[(size_t)k * nu + iu];
            cp.eta_c = (float)((eta_w - ceta) / veta);
            cp.a = (float)a;
            cp.inv_a = (a != 0.0 && (float)a != 0.0f) ? (float)(1.0 / a) : 0.0f;
            if (cp.inv_a == 0.0f) cp.a = 0.0f;
            cp.tcv = (float)(t_c / vol.vz);
            cp.kz = (float)(vol.vz / gp);
            cp.gp = (float)gp;
            cp.lxy2 = (float)(vxi * vxi * (1.0 + slope * slope));
            cp.pad = 0.0f;
        }
    }

    d.nx = vol.nx;
    d.ny = vol.ny;
    d.nz = vol.nz;
    d.nviews = nk;
    d.nu = nu;
    d.nv = nv;
    d.vx = (float)vol.vx;
    d.vy = (float)vol.vy;
    d.vz = (float)vol.vz;
    d.x0 = (float)X0;
    d.y0 = (float)Y0;
    d.z0 = (float)Z0;
    d.hx = (float)hx;
    d.hy = (float)hy;
    d.hz = (float)hz;
    d.zc = (float)(oz / vol.vz);
    d.inv_vz = (float)(1.0 / vol.vz);
    d.sdd = (float)cone.sdd;
    d.du = (float)cone.du;
    d.dv = (float)cone.dv;
    d.off_u = (float)cone.off_u;
    d.off_v = (float)cone.off_v;
    d.inv_du = (float)(1.0 / cone.du);
    d.inv_dv = (float)(1.0 / cone.dv);
    d.cu = 0.5f * (float)(nu - 1);
    d.projector = KCT_PROJECTOR_SIDDON;
    d.sid = (float)cone.sid;
    d.cv = 0.5f * (float)(nv - 1);
    d.ku = (float)(cone.sdd / cone.du);
    d.kv = (float)(cone.sdd / cone.dv);
    d.fu0 = (float)(0.5 * (nu - 1) - cone.off_u / cone.du);
    d.fv0 = (float)(0.5 * (nv - 1) - cone.off_v / cone.dv);
    d.cols = nullptr;
    d.rows = nullptr;
    d.views = nullptr;
    d.shadows = nullptr;
    d.sbx = d.sby = 0;
    return KCT_OK;
}

// The shadow table of the brick gather (ShadowParam), in double precision: for
// every view and every column of 16 x 16 voxel bricks, the detector columns
// whose pixel centres lie in the hull of its four in-plane corners' images
// widened by 0.01 column, and the extreme inverse depths of those corners.
static void shadow_table(const kct_volume_desc &vol, const kct_cone_desc &cone, std::vector<ShadowParam> &sh,
                         int &sbx, int &sby)
{
    sbx = (vol.nx + 15) / 16;
    sby = (vol.ny + 15) / 16;
    sh.assign((size_t)cone.n_views * sbx * sby, ShadowParam{});
    const double X0 = vol.cx - 0.5 * vol.nx * vol.vx, Y0 = vol.cy - 0.5 * vol.ny * vol.vy;
    const double cu = 0.5 * (cone.nu - 1);
    for (int k = 0; k < cone.n_views; ++k) {
        const double t = view_angle(cone, k);
        const double c = std::cos(t), s = std::sin(t);
        const double Sx = cone.sid * c, Sy = cone.sid * s;
        for (int by = 0; by < sby; ++by)
            for (int bx = 0; bx < sbx; ++bx) {
                const double xs[2] = {X0 + 16.0 * bx * vol.vx, X0 + std::min(16 * (bx + 1), vol.nx) * vol.vx};
                const double ys[2] = {Y0 + 16.0 * by * vol.vy, Y0 + std::min(16 * (by + 1), vol.ny) * vol.vy};
                double umin = INFINITY, umax = -INFINITY, rmin = INFINITY, rmax = -INFINITY;
                for (int cc = 0; cc < 4; ++cc) {
                    const double dx = xs[cc & 1] - Sx, dy = ys[cc >> 1] - Sy;
                    const double num = -s * dx + c * dy, den = -c * dx - s * dy;  // den > 0 (checked above)
                    const double u = (cone.sdd * num / den - cone.off_u) / cone.du + cu;
                    umin = std::min(umin, u);
                    umax = std::max(umax, u);
                    rmin = std::min(rmin, 1.0 / den);
                    rmax = std::max(rmax, 1.0 / den);
                }
                ShadowParam &p = sh[((size_t)k * sby + by) * sbx + bx];
                p.u0 = std::max(0, (int)std::ceil(umin - 0.01));
                p.u1 = std::min(cone.nu - 1, (int)std::floor(umax + 0.01));
                p.rmin = (float)rmin;
                p.rmax = (float)rmax;
            }
    }
}

kct_status geometry_build(const kct_volume_desc &vol, const kct_cone_desc &cone, Geometry *g)
{
    std::vector<ColParam> cols;
    std::vector<RowParam> rows;
    std::vector<ViewParam> views;
    kct_status st = geometry_tables(vol, cone, cols, rows, views, g->dev);
    if (st != KCT_OK) return st;
    g->vol = vol;
    g->cone = cone;
    g->cone.angles = nullptr;  // the handle does not keep the caller's pointer
    GeoDev &d = g->dev;

    std::vector<ShadowParam> shadows;
    shadow_table(vol, cone, shadows, d.sbx, d.sby);
    size_t cb = cols.size() * sizeof(ColParam), rb = rows.size() * sizeof(RowParam);
    size_t vb = views.size() * sizeof(ViewParam), sb = shadows.size() * sizeof(ShadowParam);
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    size_t total = al(cb) + al(rb) + al(vb) + al(sb);
    if (hipGetDevice(&g->device) != hipSuccess) {
        set_error("kct_geometry_create: hipGetDevice failed");
        return KCT_ERR_HIP;
    }
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, total);
    if (e != hipSuccess) {
        set_error(std::string("kct_geometry_create: hipMalloc of the ray tables failed: ") + hipGetErrorString(e));
        return KCT_ERR_HIP;
    }
    char *base = (char *)p;
    e = hipMemcpy(base, cols.data(), cb, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(base + al(cb), rows.data(), rb, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(base + al(cb) + al(rb), views.data(), vb, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(base + al(cb) + al(rb) + al(vb), shadows.data(), sb, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(p);
        set_error(std::string("kct_geometry_create: table upload failed: ") + hipGetErrorString(e));
        return KCT_ERR_HIP;
    }
    g->d_tables = p;
    g->table_bytes = total;
    d.cols = (const ColParam *)base;
    d.rows = (const RowParam *)(base + al(cb));
    d.views = (const ViewParam *)(base + al(cb) + al(rb));
    d.shadows = (const ShadowParam *)(base + al(cb) + al(rb) + al(vb));
    return KCT_OK;
}

}  // namespace kct
