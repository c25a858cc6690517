// Host side of the pbftherm C ABI: problem description, device binding and the
// drivers that enqueue the HIP kernels.  See include/pbftherm.h for the
// contract of every entry point.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "pbf_internal.h"

using namespace pbf;

struct pbf_ctx {
    std::string err;
    // mesh
    bool has_mesh = false;
    int degree = 0, nx = 0, ny = 0, nz = 0;
    double L[3] = {0, 0, 0};
    // boundary
    unsigned dmask = 0;
    double T_D = 0.0;
    // material
    bool has_material = false;
    int n_bp = 0;
    double T_bp[kMaxBp], k_bp[kMaxBp], cp_bp[kMaxBp];
    double rho = 0, T_s = 0, T_l = 0, latent = 0, phi = 1, powder_depth = 0;
    int hist_layers = 0;
    std::vector<int> powder_levels;  // [layer][qz] of the history layers
    // laser
    int laser_kind = -1;
    double radius = 0, absorptivity = 0, h_powder = 0, t_start = 0;
    std::vector<pbf_track> tracks;
    std::vector<double> track_t0, track_len;
    // FP32 reference temperature
    double Tref = 0.0;
    // device binding
    bool bound = false;
    char *ws = nullptr;
    size_t ws_bytes = 0;
    Law<double> *d_law64 = nullptr, *d_lin64 = nullptr;
    Law<float> *d_law32 = nullptr;
    double *d_slots = nullptr;
    double *d_f = nullptr, *d_C = nullptr, *d_v = nullptr, *d_partials = nullptr, *d_scal = nullptr;
    double *d_cg[8] = {};  // implicit step: y, diag, r, z, p, Ap, x, d
    bool laws_dirty = true;
    Law<double> h_law64{}, h_lin64{};
    Law<float> h_law32{};
    // kernel timing: 3 events per timed step (before cells, between, after faces)
    std::vector<hipEvent_t> tev;
    size_t tev_used = 0;
    bool timing = false;
};

namespace {

thread_local std::string g_create_err;

pbf_status fail(pbf_ctx *c, pbf_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (c) c->err = buf;
    else g_create_err = buf;
    return st;
}

#define PBF_HIP(ctx, expr)                                                                        \
    do {                                                                                          \
        hipError_t e_ = (expr);                                                                   \
        if (e_ != hipSuccess)                                                                     \
            return fail(ctx, PBF_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));         \
    } while (0)

long long nodes1(const pbf_ctx *c, int d)
{
    const int n = d == 0 ? c->nx : (d == 1 ? c->ny : c->nz);
    return (long long)c->degree * n + 1;
}
long long n_dofs(const pbf_ctx *c) { return nodes1(c, 0) * nodes1(c, 1) * nodes1(c, 2); }
long long n_cells(const pbf_ctx *c) { return (long long)c->nx * c->ny * c->nz; }
int nq1(const pbf_ctx *c) { return c->degree + 1; }
long long n_hist_cells(const pbf_ctx *c) { return (long long)c->nx * c->ny * c->hist_layers; }
long long n_hist_qp(const pbf_ctx *c)
{
    const long long q = nq1(c);
    return n_hist_cells(c) * q * q * q;
}
int ceil_div(int a, int b) { return (a + b - 1) / b; }
size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

double gauss_point(int degree, int i)
{
    return degree == 1 ? Tables<1>::gp(i) : Tables<2>::gp(i);
}

// history layers: top cell layers that hold a Gauss level within powder_depth of the top
void compute_history_layers(pbf_ctx *c)
{
    c->hist_layers = 0;
    c->powder_levels.clear();
    if (!c->has_mesh || !c->has_material) return;
    const double hz = c->L[2] / c->nz;
    const int n1 = nq1(c);
    std::vector<int> levels;
    int layers = 0;
    for (int cz = c->nz - 1; cz >= 0; --cz) {
        bool any = false;
        std::vector<int> lev(n1, 0);
        for (int qz = 0; qz < n1; ++qz) {
            const double z = (cz + gauss_point(c->degree, qz)) * hz;
            lev[qz] = (c->L[2] - z <= c->powder_depth) ? 1 : 0;
            any = any || lev[qz];
        }
        if (!any) break;
        ++layers;
        levels.insert(levels.begin(), lev.begin(), lev.end());  // bottom layer first
    }
    c->hist_layers = layers;
    c->powder_levels = levels;
}

template <typename R>
void build_law(const pbf_ctx *c, double Tref, bool linear, int crit, Law<R> &L)
{
    std::memset(&L, 0, sizeof L);
    if (linear) {
        L.n_hinge = 0;
        L.k0 = R(c->k_bp[crit]);
        L.c0 = R(c->cp_bp[crit]);
        L.Ts = R(3.0e38);
        L.Tl = R(3.0e38);
        L.inv_dT = R(0);
        L.lat = R(0);
        L.phi = R(1);
        L.rho = R(c->rho);
        return;
    }
    const int n = c->n_bp;
    L.k0 = R(c->k_bp[0]);
    L.c0 = R(c->cp_bp[0]);
    if (n >= 2) {
        double sk_prev = 0.0, sc_prev = 0.0;
        for (int i = 0; i < n; ++i) {
            double sk = 0.0, sc = 0.0;  // slope of the segment starting at b_i
            if (i < n - 1) {
                sk = (c->k_bp[i + 1] - c->k_bp[i]) / (c->T_bp[i + 1] - c->T_bp[i]);
                sc = (c->cp_bp[i + 1] - c->cp_bp[i]) / (c->T_bp[i + 1] - c->T_bp[i]);
            }
            L.b[i] = R(c->T_bp[i] - Tref);
            L.dk[i] = R(sk - sk_prev);
            L.dc[i] = R(sc - sc_prev);
            sk_prev = sk;
            sc_prev = sc;
        }
        L.n_hinge = n;
    }
    L.Ts = R(c->T_s - Tref);
    L.Tl = R(c->T_l - Tref);
    L.inv_dT = R(1.0 / (c->T_l - c->T_s));
    L.lat = R(c->latent / (c->T_l - c->T_s));
    L.phi = R(c->phi);
    L.rho = R(c->rho);
}

int critical_breakpoint(const pbf_ctx *c)
{
    int best = 0;
    for (int i = 1; i < c->n_bp; ++i)
        if (c->k_bp[i] / c->cp_bp[i] > c->k_bp[best] / c->cp_bp[best]) best = i;
    return best;
}

struct Beam {
    bool on;
    double xb, yb, W;
    int track;
};

// beam centre and effective power at time t (tracks in order, each at its speed)
Beam beam_at(const pbf_ctx *c, double t)
{
    Beam b{false, 0, 0, 0, -1};
    if (c->laser_kind < 0 || c->tracks.empty() || t < c->t_start) return b;
    for (size_t k = 0; k < c->tracks.size(); ++k) {
        const pbf_track &tr = c->tracks[k];
        const double len = c->track_len[k];
        const double t0 = c->track_t0[k];
        if (t < t0 + len / tr.speed) {
            const double s = (t - t0) * tr.speed / len;
            b.on = true;
            b.xb = tr.x0[0] + s * (tr.x1[0] - tr.x0[0]);
            b.yb = tr.x0[1] + s * (tr.x1[1] - tr.x0[1]);
            b.W = c->absorptivity * tr.power;
            b.track = (int)k;
            return b;
        }
    }
    return b;
}

// Cell layers per z-segment of a column workgroup: minimizes the makespan
// (rounds of resident workgroups x layers per workgroup), two workgroups per CU
// on 256 CUs, preferring longer segments (fewer segment faces) on ties.
int segment_length(const pbf_ctx *c, int ty, int resident_per_cu)
{
    const long long cols = (long long)ceil_div(c->nx, kTX) * ceil_div(c->ny, ty);
    const long long slots = 256LL * resident_per_cu;
    int best = c->nz;
    long long best_cost = -1;
    for (int S = std::min(c->nz, 32); S >= 1; --S) {
        const long long blocks = cols * ceil_div(c->nz, S);
        const long long cost = ((blocks + slots - 1) / slots) * S;
        if (best_cost < 0 || cost < best_cost) {
            best_cost = cost;
            best = S;
        }
    }
    return best;
}

// Column geometry of a cell kernel with columns of 16 x ty cells and the given
// number of resident workgroups per CU (explicit kernels by default).
HaloParams geometry(const pbf_ctx *c, int ty = -1, int resident = -1)
{
    if (ty < 0) {
        ty = column_height();
        resident = resident_columns_per_cu(ty);
    }
    HaloParams h{};
    const int P = c->degree;
    const int S = segment_length(c, ty, resident);
    h.NX = (int)nodes1(c, 0);
    h.NY = (int)nodes1(c, 1);
    h.NZ = (int)nodes1(c, 2);
    h.SX = P * kTX;
    h.SY = P * ty;
    h.SZ = P * S;
    h.MX = ceil_div(c->nx, kTX);
    h.MY = ceil_div(c->ny, ty);
    h.MZ = ceil_div(c->nz, S);
    h.GX = (long long)(h.MX - 1) * h.NY * h.NZ;
    h.GY = (long long)h.NX * (h.MY - 1) * h.NZ;
    h.GZ = (long long)h.NX * h.NY * (h.MZ - 1);
    h.T_D = c->T_D;
    h.dmask = c->dmask;
    h.slots = c->d_slots;
    h.nlaw = c->d_law64;
    h.P = P;
    h.hx = c->L[0] / c->nx;
    h.hy = c->L[1] / c->ny;
    h.hz = c->L[2] / c->nz;
    return h;
}

template <typename R>
CellParams<R> cell_params(const pbf_ctx *c, const Law<R> *law, bool history)
{
    CellParams<R> p{};
    const HaloParams h = geometry(c);
    p.nx = c->nx;
    p.ny = c->ny;
    p.nz = c->nz;
    p.NX = h.NX;
    p.NY = h.NY;
    p.NZ = h.NZ;
    p.MX = h.MX;
    p.MY = h.MY;
    p.MZ = h.MZ;
    p.ntiles = h.MX * h.MY * h.MZ;
    p.tiles_per_xcd = ceil_div(p.ntiles, 8);
    p.seg_len = h.SZ / c->degree;
    p.hist_cz0 = history ? c->nz - c->hist_layers : c->nz;
    p.n_hist_cells = (int)n_hist_cells(c);
    p.hx = c->L[0] / c->nx;
    p.hy = c->L[1] / c->ny;
    p.hz = c->L[2] / c->nz;
    p.Lz = c->L[2];
    p.detJ = R(p.hx * p.hy * p.hz);
    p.ih2x = R(1.0 / (p.hx * p.hx));
    p.ih2y = R(1.0 / (p.hy * p.hy));
    p.ih2z = R(1.0 / (p.hz * p.hz));
    p.T_D = c->T_D;
    p.Tref = std::is_same<R, double>::value ? 0.0 : c->Tref;
    p.dmask = c->dmask;
    p.slots = c->d_slots;
    p.law = law;
    p.nlaw = c->d_law64;
    p.laser_on = 0;
    p.laser_kind = c->laser_kind;
    const double depth_cells = (c->L[2] - c->h_powder) / p.hz;
    p.src_cz0 = std::max(0, (int)std::floor(depth_cells) - 1);
    p.h_powder = c->h_powder;
    p.two_over_R2 = c->radius > 0 ? 2.0 / (c->radius * c->radius) : 0.0;
    return p;
}

template <typename R>
void set_beam(const pbf_ctx *c, CellParams<R> &p, double t)
{
    const Beam b = beam_at(c, t);
    p.laser_on = b.on ? 1 : 0;
    p.xb = b.xb;
    p.yb = b.yb;
    const double PI = 3.14159265358979323846;
    const double R2 = c->radius * c->radius;
    if (c->laser_kind == 1) p.src_amp = 2.0 * b.W / (PI * R2 * c->h_powder);
    else p.src_amp = 2.0 * b.W / (PI * R2);
}

pbf_status check_bound(pbf_ctx *c)
{
    if (!c->has_mesh) return fail(c, PBF_ESTATE, "no mesh: call pbf_mesh_box first");
    if (!c->has_material) return fail(c, PBF_ESTATE, "no material: call pbf_set_material first");
    if (!c->bound) return fail(c, PBF_ESTATE, "no device workspace: call pbf_bind_device first");
    return PBF_OK;
}

pbf_status upload_laws(pbf_ctx *c, hipStream_t s)
{
    if (!c->laws_dirty) return PBF_OK;
    build_law<double>(c, 0.0, false, 0, c->h_law64);
    build_law<float>(c, c->Tref, false, 0, c->h_law32);
    build_law<double>(c, 0.0, true, critical_breakpoint(c), c->h_lin64);
    PBF_HIP(c, hipMemcpyAsync(c->d_law64, &c->h_law64, sizeof(Law<double>), hipMemcpyHostToDevice, s));
    PBF_HIP(c, hipMemcpyAsync(c->d_law32, &c->h_law32, sizeof(Law<float>), hipMemcpyHostToDevice, s));
    PBF_HIP(c, hipMemcpyAsync(c->d_lin64, &c->h_lin64, sizeof(Law<double>), hipMemcpyHostToDevice, s));
    PBF_HIP(c, hipStreamSynchronize(s));
    c->laws_dirty = false;
    return PBF_OK;
}

// one operator pass: MODE 0 explicit step Tin -> Tout, MODE 1 assemble into f, C
pbf_status operator_pass(pbf_ctx *c, int mode, int precision, bool linear, const double *Tin,
                         double *Tout, double *f, double *C, double *rc, double t, double dt,
                         hipStream_t s)
{
    CellParams<double> pd{};
    CellParams<float> pf{};
    if (precision == PBF_PREC_FP64) {
        pd = cell_params<double>(c, linear ? c->d_lin64 : c->d_law64, !linear);
        pd.Tin = Tin;
        pd.Tout = Tout;
        pd.fout = f;
        pd.Cout = C;
        pd.hist = rc;
        pd.dt = dt;
        if (!linear) set_beam(c, pd, t);
    } else {
        pf = cell_params<float>(c, c->d_law32, true);
        pf.Tin = Tin;
        pf.Tout = Tout;
        pf.fout = f;
        pf.Cout = C;
        pf.hist = rc;
        pf.dt = dt;
        set_beam(c, pf, t);
    }
    if (linear) pd.nlaw = c->d_lin64;
    const bool timed = c->timing && mode == 0 && c->tev_used + 3 <= c->tev.size();
    if (timed) PBF_HIP(c, hipEventRecord(c->tev[c->tev_used], s));
    PBF_HIP(c, launch_cells(c->degree, precision, mode, column_height(), pd, pf, s));
    if (timed) PBF_HIP(c, hipEventRecord(c->tev[c->tev_used + 1], s));
    HaloParams h = geometry(c);
    if (linear) h.nlaw = c->d_lin64;
    h.Tin = Tin;
    h.Tout = Tout;
    h.fout = f;
    h.Cout = C;
    h.dt = dt;
    PBF_HIP(c, launch_halo(mode, h, s));
    if (timed) {
        PBF_HIP(c, hipEventRecord(c->tev[c->tev_used + 2], s));
        c->tev_used += 3;
    }
    return PBF_OK;
}

// Picard-operator parameters (apply or diagonal) for C(Tc)/dt + K(Tk)
PicardParams picard_params(const pbf_ctx *c, const HaloParams &h, const double *Tc, const double *Tk,
                           const double *x1, const double *x2, double *y, const double *rc,
                           double dt, const Beam *src)
{
    PicardParams q{};
    q.Tc = Tc;
    q.Tk = Tk;
    q.x1 = x1;
    q.x2 = x2;
    q.yout = y;
    q.hist = rc;
    q.slots = c->d_slots;
    q.nx = c->nx;
    q.ny = c->ny;
    q.nz = c->nz;
    q.NX = h.NX;
    q.NY = h.NY;
    q.NZ = h.NZ;
    q.MX = h.MX;
    q.MY = h.MY;
    q.MZ = h.MZ;
    q.ntiles = h.MX * h.MY * h.MZ;
    q.tiles_per_xcd = ceil_div(q.ntiles, 8);
    q.seg_len = h.SZ / c->degree;
    q.hist_cz0 = c->nz - c->hist_layers;
    q.n_hist_cells = (int)n_hist_cells(c);
    q.hx = c->L[0] / c->nx;
    q.hy = c->L[1] / c->ny;
    q.hz = c->L[2] / c->nz;
    q.Lz = c->L[2];
    q.detJ = q.hx * q.hy * q.hz;
    q.ih2x = 1.0 / (q.hx * q.hx);
    q.ih2y = 1.0 / (q.hy * q.hy);
    q.ih2z = 1.0 / (q.hz * q.hz);
    q.inv_dt = 1.0 / dt;
    q.dmask = c->dmask;
    q.laser_kind = c->laser_kind;
    const double depth_cells = (c->L[2] - c->h_powder) / q.hz;
    q.src_cz0 = std::max(0, (int)std::floor(depth_cells) - 1);
    q.h_powder = c->h_powder;
    q.two_over_R2 = c->radius > 0 ? 2.0 / (c->radius * c->radius) : 0.0;
    q.src_on = 0;
    if (src && src->on) {
        const double PI = 3.14159265358979323846, R2 = c->radius * c->radius;
        q.src_on = 1;
        q.xb = src->xb;
        q.yb = src->yb;
        q.src_amp = c->laser_kind == 1 ? 2.0 * src->W / (PI * R2 * c->h_powder) : 2.0 * src->W / (PI * R2);
    }
    q.law = c->d_law64;
    return q;
}

}  // namespace

extern "C" {

pbf_status pbf_create(pbf_ctx **out)
{
    if (!out) return fail(nullptr, PBF_EINVAL, "pbf_create: out is NULL");
    *out = new (std::nothrow) pbf_ctx();
    if (!*out) return fail(nullptr, PBF_ENOMEM, "pbf_create: out of host memory");
    return PBF_OK;
}

void pbf_destroy(pbf_ctx *ctx)
{
    if (!ctx) return;
    for (hipEvent_t e : ctx->tev) (void)hipEventDestroy(e);
    delete ctx;
}

const char *pbf_last_error(const pbf_ctx *ctx)
{
    return ctx ? ctx->err.c_str() : g_create_err.c_str();
}

pbf_status pbf_mesh_box(pbf_ctx *c, int degree, int nx, int ny, int nz, double Lx, double Ly,
                        double Lz)
{
    if (!c) return fail(nullptr, PBF_EINVAL, "pbf_mesh_box: ctx is NULL");
    if (degree != 1 && degree != 2) return fail(c, PBF_EMESH, "degree %d not supported (1 or 2)", degree);
    if (nx < 1 || ny < 1 || nz < 1) return fail(c, PBF_EINVAL, "cell counts must be >= 1");
    if (!(Lx > 0 && Ly > 0 && Lz > 0)) return fail(c, PBF_EINVAL, "box lengths must be > 0");
    const long long NX = (long long)degree * nx + 1, NY = (long long)degree * ny + 1,
                    NZ = (long long)degree * nz + 1;
    if (NX > (1 << 30) || NY > (1 << 30) || NZ > (1 << 30) || NX * NY * NZ > (1LL << 40))
        return fail(c, PBF_EMESH, "mesh too large");
    c->has_mesh = true;
    c->degree = degree;
    c->nx = nx;
    c->ny = ny;
    c->nz = nz;
    c->L[0] = Lx;
    c->L[1] = Ly;
    c->L[2] = Lz;
    c->bound = false;
    c->laws_dirty = true;
    compute_history_layers(c);
    return PBF_OK;
}

pbf_status pbf_mesh_info(const pbf_ctx *c, int64_t *nd, int64_t *nc, int64_t *nq, int64_t *nhl,
                         int64_t *nhc, int64_t *nhq)
{
    if (!c) return fail(nullptr, PBF_EINVAL, "pbf_mesh_info: ctx is NULL");
    if (!c->has_mesh) return fail(const_cast<pbf_ctx *>(c), PBF_ESTATE, "no mesh");
    const long long q = nq1(c);
    if (nd) *nd = n_dofs(c);
    if (nc) *nc = n_cells(c);
    if (nq) *nq = n_cells(c) * q * q * q;
    if (nhl) *nhl = c->hist_layers;
    if (nhc) *nhc = n_hist_cells(c);
    if (nhq) *nhq = n_hist_qp(c);
    return PBF_OK;
}

pbf_status pbf_set_dirichlet(pbf_ctx *c, unsigned face_mask, double T_D)
{
    if (!c) return fail(nullptr, PBF_EINVAL, "pbf_set_dirichlet: ctx is NULL");
    if (face_mask > 63u) return fail(c, PBF_EINVAL, "face mask must use bits 0..5");
    if (!std::isfinite(T_D)) return fail(c, PBF_EINVAL, "T_D must be finite");
    c->dmask = face_mask;
    c->T_D = T_D;
    return PBF_OK;
}

pbf_status pbf_set_material(pbf_ctx *c, const pbf_material *m)
{
    if (!c || !m) return fail(c, PBF_EINVAL, "pbf_set_material: NULL argument");
    if (m->n_bp < 1 || m->n_bp > kMaxBp) return fail(c, PBF_EINVAL, "n_bp must be in [1,%d]", kMaxBp);
    if (!m->T_bp || !m->k_bp || !m->cp_bp) return fail(c, PBF_EINVAL, "NULL breakpoint table");
    for (int i = 0; i < m->n_bp; ++i) {
        if (!std::isfinite(m->T_bp[i]) || !(m->k_bp[i] > 0) || !(m->cp_bp[i] > 0))
            return fail(c, PBF_EINVAL, "breakpoint %d: need finite T and k, c_p > 0", i);
        if (i > 0 && !(m->T_bp[i] > m->T_bp[i - 1]))
            return fail(c, PBF_EINVAL, "breakpoints must be strictly increasing");
    }
    if (!(m->rho > 0)) return fail(c, PBF_EINVAL, "rho must be > 0");
    if (!(m->T_l > m->T_s)) return fail(c, PBF_EINVAL, "need T_l > T_s");
    if (!(m->latent >= 0)) return fail(c, PBF_EINVAL, "latent heat must be >= 0");
    if (!(m->powder_k_factor > 0 && m->powder_k_factor <= 1))
        return fail(c, PBF_EINVAL, "powder_k_factor must be in (0,1]");
    if (!(m->powder_depth >= 0)) return fail(c, PBF_EINVAL, "powder_depth must be >= 0");
    c->n_bp = m->n_bp;
    for (int i = 0; i < m->n_bp; ++i) {
        c->T_bp[i] = m->T_bp[i];
        c->k_bp[i] = m->k_bp[i];
        c->cp_bp[i] = m->cp_bp[i];
    }
    c->rho = m->rho;
    c->T_s = m->T_s;
    c->T_l = m->T_l;
    c->latent = m->latent;
    c->phi = m->powder_k_factor;
    c->powder_depth = m->powder_depth;
    c->has_material = true;
    c->laws_dirty = true;
    const int old_layers = c->hist_layers;
    compute_history_layers(c);
    if (c->bound && c->hist_layers != old_layers) c->bound = false;  // sizes changed
    return PBF_OK;
}

pbf_status pbf_set_laser(pbf_ctx *c, const pbf_laser *l)
{
    if (!c || !l) return fail(c, PBF_EINVAL, "pbf_set_laser: NULL argument");
    if (l->kind < -1 || l->kind > 1) return fail(c, PBF_EINVAL, "laser kind must be -1, 0 or 1");
    if (l->n_tracks < 0 || l->n_tracks > 4096) return fail(c, PBF_EINVAL, "n_tracks out of range");
    if (l->n_tracks > 0 && !l->tracks) return fail(c, PBF_EINVAL, "NULL track array");
    if (l->kind >= 0 && !(l->radius > 0)) return fail(c, PBF_EINVAL, "radius must be > 0");
    if (l->kind == 1 && !(l->h_powder > 0)) return fail(c, PBF_EINVAL, "h_powder must be > 0");
    std::vector<pbf_track> tr(l->tracks, l->tracks + l->n_tracks);
    std::vector<double> t0(tr.size()), len(tr.size());
    double tk = l->t_start;
    for (size_t k = 0; k < tr.size(); ++k) {
        const double dx = tr[k].x1[0] - tr[k].x0[0], dy = tr[k].x1[1] - tr[k].x0[1],
                     dz = tr[k].x1[2] - tr[k].x0[2];
        len[k] = std::sqrt(dx * dx + dy * dy + dz * dz);
        if (!(len[k] > 0) || !(tr[k].speed > 0) || !(tr[k].power >= 0))
            return fail(c, PBF_EINVAL, "track %zu: need length > 0, speed > 0, power >= 0", k);
        t0[k] = tk;
        tk += len[k] / tr[k].speed;
    }
    c->laser_kind = l->kind;
    c->radius = l->radius;
    c->absorptivity = l->absorptivity;
    c->h_powder = l->h_powder;
    c->t_start = l->t_start;
    c->tracks = tr;
    c->track_t0 = t0;
    c->track_len = len;
    return PBF_OK;
}

pbf_status pbf_set_track_powers(pbf_ctx *c, const double *power, double absorptivity)
{
    if (!c || (!power && !c->tracks.empty())) return fail(c, PBF_EINVAL, "NULL argument");
    for (size_t k = 0; k < c->tracks.size(); ++k)
        if (!(power[k] >= 0)) return fail(c, PBF_EINVAL, "power %zu must be >= 0", k);
    for (size_t k = 0; k < c->tracks.size(); ++k) c->tracks[k].power = power[k];
    c->absorptivity = absorptivity;
    return PBF_OK;
}

pbf_status pbf_workspace_bytes(const pbf_ctx *c, size_t *bytes)
{
    if (!c || !bytes) return fail(const_cast<pbf_ctx *>(c), PBF_EINVAL, "NULL argument");
    if (!c->has_mesh) return fail(const_cast<pbf_ctx *>(c), PBF_ESTATE, "no mesh");
    const size_t N = (size_t)n_dofs(c);
    size_t b = 0;
    b += align256(sizeof(Law<double>)) * 2 + align256(sizeof(Law<float>));
    b += align256(8 * N * sizeof(double));        // parity slots
    b += 11 * align256(N * sizeof(double));       // f, C, v; implicit: y, diag, r, z, p, Ap, x, d
    b += align256(kRedBlocks * 4 * sizeof(double)); // reduction partials
    b += align256(64 * sizeof(double));           // device scalars
    *bytes = b;
    return PBF_OK;
}

pbf_status pbf_bind_device(pbf_ctx *c, void *workspace, size_t bytes, void *stream)
{
    if (!c) return fail(nullptr, PBF_EINVAL, "ctx is NULL");
    size_t need = 0;
    pbf_status st = pbf_workspace_bytes(c, &need);
    if (st) return st;
    if (!workspace) return fail(c, PBF_EINVAL, "workspace is NULL");
    if (((uintptr_t)workspace & 255) != 0) return fail(c, PBF_EINVAL, "workspace must be 256-byte aligned");
    if (bytes < need) return fail(c, PBF_ENOMEM, "workspace too small: %zu < %zu bytes", bytes, need);
    const size_t N = (size_t)n_dofs(c);
    char *p = (char *)workspace;
    c->d_law64 = (Law<double> *)p;
    p += align256(sizeof(Law<double>));
    c->d_lin64 = (Law<double> *)p;
    p += align256(sizeof(Law<double>));
    c->d_law32 = (Law<float> *)p;
    p += align256(sizeof(Law<float>));
    c->d_slots = (double *)p;
    p += align256(8 * N * sizeof(double));
    c->d_f = (double *)p;
    p += align256(N * sizeof(double));
    c->d_C = (double *)p;
    p += align256(N * sizeof(double));
    c->d_v = (double *)p;
    p += align256(N * sizeof(double));
    for (int k = 0; k < 8; ++k) {
        c->d_cg[k] = (double *)p;
        p += align256(N * sizeof(double));
    }
    c->d_partials = (double *)p;
    p += align256(kRedBlocks * 4 * sizeof(double));
    c->d_scal = (double *)p;
    c->ws = (char *)workspace;
    c->ws_bytes = bytes;
    c->bound = true;
    c->laws_dirty = true;
    if (c->has_material) return upload_laws(c, (hipStream_t)stream);
    return PBF_OK;
}

pbf_status pbf_init_state(pbf_ctx *c, double T0, double *T, double *rc, void *stream)
{
    if (!c) return fail(nullptr, PBF_EINVAL, "ctx is NULL");
    pbf_status st = check_bound(c);
    if (st) return st;
    if (!T) return fail(c, PBF_EINVAL, "T is NULL");
    if (n_hist_qp(c) > 0 && !rc) return fail(c, PBF_EINVAL, "rc is NULL but the mesh has history");
    if (!std::isfinite(T0)) return fail(c, PBF_EINVAL, "T0 must be finite");
    hipStream_t s = (hipStream_t)stream;
    if (c->Tref != T0) {
        c->Tref = T0;
        c->laws_dirty = true;
    }
    if ((st = upload_laws(c, s))) return st;
    PBF_HIP(c, launch_fill(T, T0, n_dofs(c), s));
    PBF_HIP(c, launch_init_dirichlet(T, geometry(c), c->T_D, s));
    if (n_hist_qp(c) > 0)
        PBF_HIP(c, launch_init_history(rc, (int)n_hist_cells(c), nq1(c), c->powder_levels.data(),
                                       c->hist_layers, c->nx, c->ny, s));
    return PBF_OK;
}

pbf_status pbf_explicit_steps(pbf_ctx *c, double *T, double *T_tmp, double *rc, double t0,
                              double dt, int n_steps, int precision, void *stream)
{
    if (!c) return fail(nullptr, PBF_EINVAL, "ctx is NULL");
    pbf_status st = check_bound(c);
    if (st) return st;
    if (!T || !T_tmp || T == T_tmp) return fail(c, PBF_EINVAL, "T and T_tmp must be distinct device arrays");
    if (n_hist_qp(c) > 0 && !rc) return fail(c, PBF_EINVAL, "rc is NULL but the mesh has history");
    if (n_steps < 0) return fail(c, PBF_EINVAL, "n_steps must be >= 0");
    if (!(dt > 0) || !std::isfinite(t0)) return fail(c, PBF_EINVAL, "need dt > 0 and finite t0");
    if (precision != PBF_PREC_FP64 && precision != PBF_PREC_FP32)
        return fail(c, PBF_EINVAL, "precision must be 64 or 32");
    hipStream_t s = (hipStream_t)stream;
    if ((st = upload_laws(c, s))) return st;
    double *cur = T, *nxt = T_tmp;
    for (int n = 0; n < n_steps; ++n) {
        const double t = t0 + n * dt;
        st = operator_pass(c, 0, precision, false, cur, nxt, nullptr, nullptr, rc, t, dt, s);
        if (st) return st;
        std::swap(cur, nxt);
    }
    if (cur != T) PBF_HIP(c, hipMemcpyAsync(T, cur, n_dofs(c) * sizeof(double), hipMemcpyDeviceToDevice, s));
    return PBF_OK;
}

pbf_status pbf_assemble(pbf_ctx *c, const double *T, double *rc, double t, double *f, double *C,
                        int precision, void *stream)
{
    if (!c) return fail(nullptr, PBF_EINVAL, "ctx is NULL");
    pbf_status st = check_bound(c);
    if (st) return st;
    if (!T || !f || !C) return fail(c, PBF_EINVAL, "NULL device array");
    if (n_hist_qp(c) > 0 && !rc) return fail(c, PBF_EINVAL, "rc is NULL but the mesh has history");
    if (precision != PBF_PREC_FP64 && precision != PBF_PREC_FP32)
        return fail(c, PBF_EINVAL, "precision must be 64 or 32");
    hipStream_t s = (hipStream_t)stream;
    if ((st = upload_laws(c, s))) return st;
    return operator_pass(c, 1, precision, false, T, nullptr, f, C, rc, t, 0.0, s);
}

pbf_status pbf_stability_lambda(pbf_ctx *c, const double *v0, int iters, double *lambda_max,
                                void *stream)
{
    if (!c) return fail(nullptr, PBF_EINVAL, "ctx is NULL");
    pbf_status st = check_bound(c);
    if (st) return st;
    if (!v0 || !lambda_max) return fail(c, PBF_EINVAL, "NULL argument");
    if (iters < 1) return fail(c, PBF_EINVAL, "iters must be >= 1");
    hipStream_t s = (hipStream_t)stream;
    if ((st = upload_laws(c, s))) return st;
    const long long N = n_dofs(c);
    const HaloParams g = geometry(c);
    PBF_HIP(c, hipMemcpyAsync(c->d_v, v0, N * sizeof(double), hipMemcpyDeviceToDevice, s));
    PBF_HIP(c, launch_init_dirichlet(c->d_v, g, 0.0, s));
    for (int it = 0; it < iters; ++it) {
        st = operator_pass(c, 1, PBF_PREC_FP64, true, c->d_v, nullptr, c->d_f, c->d_C, nullptr, 0.0,
                           0.0, s);
        if (st) return st;
        PBF_HIP(c, launch_power_dots(c->d_f, c->d_C, c->d_v, c->d_partials, c->d_scal, g, N, s));
        PBF_HIP(c, launch_power_update(c->d_f, c->d_C, c->d_v, c->d_partials, c->d_scal, g, N, s));
        PBF_HIP(c, launch_power_scale(c->d_v, c->d_scal, N, s));
    }
    double sc[2];
    PBF_HIP(c, hipMemcpyAsync(sc, c->d_scal, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
    PBF_HIP(c, hipStreamSynchronize(s));
    *lambda_max = sc[0] / sc[1];
    return PBF_OK;
}

pbf_status pbf_implicit_step(pbf_ctx *c, const double *T_n, double *T_out, double *rc, double t,
                             double dt, double cg_rtol, int cg_max_it, double picard_tol,
                             int picard_max_it, int *cg_iters_total, int *picard_iters,
                             double *final_rel_res, void *stream)
{
    if (!c) return fail(nullptr, PBF_EINVAL, "ctx is NULL");
    pbf_status st = check_bound(c);
    if (st) return st;
    if (!T_n || !T_out || T_n == T_out) return fail(c, PBF_EINVAL, "T_n and T_out must be distinct device arrays");
    if (n_hist_qp(c) > 0 && !rc) return fail(c, PBF_EINVAL, "rc is NULL but the mesh has history");
    if (!(dt > 0) || !std::isfinite(t)) return fail(c, PBF_EINVAL, "need dt > 0 and finite t");
    if (!(cg_rtol > 0) || cg_max_it < 1 || !(picard_tol > 0) || picard_max_it < 1)
        return fail(c, PBF_EINVAL, "tolerances must be > 0 and iteration limits >= 1");
    hipStream_t s = (hipStream_t)stream;
    if ((st = upload_laws(c, s))) return st;
    const long long N = n_dofs(c);
    const HaloParams ge = geometry(c);  // explicit-kernel geometry (history commit)
    const HaloParams hp = geometry(c, picard_column_height(), 3);
    double *y = c->d_cg[0], *diag = c->d_cg[1], *r = c->d_cg[2], *z = c->d_cg[3], *p = c->d_cg[4],
           *Ap = c->d_cg[5], *x = c->d_cg[6], *d = c->d_cg[7];
    double *Ti = T_out;
    PBF_HIP(c, hipMemcpyAsync(Ti, T_n, N * sizeof(double), hipMemcpyDeviceToDevice, s));
    PBF_HIP(c, launch_init_dirichlet(Ti, ge, c->T_D, s));
    const Beam bm = beam_at(c, t + dt);
    int total = 0, it = 0;
    bool cg_fail = false, converged = false;
    double last_rel = 0.0;
    double hs[8];
    for (it = 0; it < picard_max_it;) {
        // residual R(T^i) = C(T_n)(T^i - T_n)/dt + K(T^i) T^i - f_vol, and diag(A(T^i))
        PBF_HIP(c, launch_sub(d, Ti, T_n, N, s));
        PicardParams qa = picard_params(c, hp, T_n, Ti, d, Ti, y, rc, dt, &bm);
        PBF_HIP(c, launch_picard(c->degree, 0, qa, hp, s));
        PicardParams qd = picard_params(c, hp, T_n, Ti, nullptr, nullptr, diag, rc, dt, nullptr);
        PBF_HIP(c, launch_picard(c->degree, 1, qd, hp, s));
        PBF_HIP(c, launch_cg_start(y, diag, r, z, p, x, c->d_partials, c->d_scal, ge, N, s));
        PBF_HIP(c, hipMemcpyAsync(hs, c->d_scal + CG_RZ0, 6 * sizeof(double), hipMemcpyDeviceToHost, s));
        PBF_HIP(c, hipStreamSynchronize(s));
        const double bn = std::sqrt(hs[CG_BN2 - CG_RZ0]);
        double rr = hs[CG_RR - CG_RZ0];
        int k = 0, rz_old = CG_RZ0;
        last_rel = bn > 0 ? std::sqrt(rr) / bn : 0.0;
        PicardParams qp = picard_params(c, hp, T_n, Ti, p, p, Ap, rc, dt, nullptr);
        while (bn > 0 && std::sqrt(rr) > cg_rtol * bn && k < cg_max_it) {
            PBF_HIP(c, launch_picard(c->degree, 0, qp, hp, s));
            PBF_HIP(c, launch_cg_pap(p, Ap, c->d_partials, c->d_scal, N, s));
            PBF_HIP(c, launch_cg_update(x, r, z, p, Ap, diag, c->d_partials, c->d_scal, rz_old, N, s));
            PBF_HIP(c, hipMemcpyAsync(&rr, c->d_scal + CG_RR, sizeof(double), hipMemcpyDeviceToHost, s));
            PBF_HIP(c, hipStreamSynchronize(s));
            const int rz_new = rz_old == CG_RZ0 ? CG_RZ1 : CG_RZ0;
            PBF_HIP(c, launch_cg_direction(p, z, c->d_scal, rz_old, rz_new, N, s));
            rz_old = rz_new;
            ++k;
            last_rel = std::sqrt(rr) / bn;
        }
        total += k;
        if (bn > 0 && std::sqrt(rr) > cg_rtol * bn) cg_fail = true;
        PBF_HIP(c, launch_picard_update(Ti, x, c->d_partials, c->d_scal, ge, N, s));
        double dmax = 0.0;
        PBF_HIP(c, hipMemcpyAsync(&dmax, c->d_scal + CG_DMAX, sizeof(double), hipMemcpyDeviceToHost, s));
        PBF_HIP(c, hipStreamSynchronize(s));
        ++it;
        if (!std::isfinite(dmax)) return fail(c, PBF_ENONFINITE, "non-finite Picard update");
        if (dmax <= picard_tol) {
            converged = true;
            break;
        }
    }
    // commit the consolidated fraction: r = max(r, g(T_{n+1}))
    st = operator_pass(c, 1, PBF_PREC_FP64, false, Ti, nullptr, c->d_f, c->d_C, rc, t + dt, 0.0, s);
    if (st) return st;
    if (cg_iters_total) *cg_iters_total = total;
    if (picard_iters) *picard_iters = it;
    if (final_rel_res) *final_rel_res = last_rel;
    if (cg_fail) return fail(c, PBF_ENOCONV, "CG did not reach the relative tolerance %g", cg_rtol);
    if (!converged) return fail(c, PBF_ENOCONV, "Picard did not converge in %d iterations", picard_max_it);
    return PBF_OK;
}

pbf_status pbf_timing_begin(pbf_ctx *c, int max_steps)
{
    if (!c) return fail(nullptr, PBF_EINVAL, "ctx is NULL");
    if (max_steps < 1 || max_steps > (1 << 22)) return fail(c, PBF_EINVAL, "max_steps out of range");
    for (hipEvent_t e : c->tev) (void)hipEventDestroy(e);
    c->tev.assign((size_t)max_steps * 3, nullptr);
    for (auto &e : c->tev) PBF_HIP(c, hipEventCreate(&e));
    c->tev_used = 0;
    c->timing = true;
    return PBF_OK;
}

pbf_status pbf_timing_end(pbf_ctx *c, double *cell_ms, double *face_ms, int64_t *n_steps)
{
    if (!c) return fail(nullptr, PBF_EINVAL, "ctx is NULL");
    if (!c->timing) return fail(c, PBF_ESTATE, "timing was not started");
    c->timing = false;
    double a = 0.0, b = 0.0;
    const size_t n = c->tev_used / 3;
    if (n > 0) PBF_HIP(c, hipEventSynchronize(c->tev[c->tev_used - 1]));
    for (size_t k = 0; k < n; ++k) {
        float t1 = 0.f, t2 = 0.f;
        PBF_HIP(c, hipEventElapsedTime(&t1, c->tev[3 * k], c->tev[3 * k + 1]));
        PBF_HIP(c, hipEventElapsedTime(&t2, c->tev[3 * k + 1], c->tev[3 * k + 2]));
        a += t1;
        b += t2;
    }
    for (hipEvent_t e : c->tev) (void)hipEventDestroy(e);
    c->tev.clear();
    c->tev_used = 0;
    if (cell_ms) *cell_ms = n ? a / n : 0.0;
    if (face_ms) *face_ms = n ? b / n : 0.0;
    if (n_steps) *n_steps = (int64_t)n;
    return PBF_OK;
}

}  // extern "C"
