// Host side of the pbftherm C ABI: problem description, device binding and the
// drivers that enqueue the HIP kernels.  See include/pbftherm.h for the
// contract of every entry point.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
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
    // radiation and evaporation on the free top surface (law pointer set per pass)
    SurfaceLoss re{};
    // FP32 reference temperature
    double Tref = 0.0;
    double T_init = 0.0;  // initial temperature (pbf_init_state): activated dofs of a growing octree
    // device binding
    bool bound = false;
    char *ws = nullptr;
    size_t ws_bytes = 0;
    Law<double> *d_law64 = nullptr, *d_lin64 = nullptr, *d_zero64 = nullptr;
    Law<float> *d_law32 = nullptr;
    double *d_slots = nullptr;
    double *d_f = nullptr, *d_C = nullptr, *d_v = nullptr, *d_partials = nullptr, *d_scal = nullptr;
    double *d_cg[8] = {};  // implicit step: y, diag, r, z, p, Ap, x, d
    double *d_tiles = nullptr;  // adjoint: per-tile source sensitivities
    double *d_coef = nullptr;   // implicit step (boxes): per-point coefficients of the CG applies
    int *d_probe_cell = nullptr;
    double *d_probe_xi = nullptr, *d_probe_target = nullptr;
    bool laws_dirty = true;
    // probes: containing cell, reference coordinates and target of each point
    std::vector<int> probe_cell;
    std::vector<double> probe_xi, probe_target;
    bool probes_dirty = false;
    // growing box (layer activation): nz and L[2] are the active cell layers and
    // height; nz_full and Lz_full the allocated box (state arrays, workspace)
    bool growing = false;
    int nz_full = 0;
    double Lz_full = 0.0;
    // octree mesh (when octree is set, nx, ny, nz are the coarse cells)
    bool octree = false;
    bool oct_flags_dirty = false;  // Dirichlet flags / history leaves changed since the upload
    OctMesh oct;
    OctDev od{};
    struct {                // remesh prepared by pbf_octree_remesh_bytes
        bool ready = false;
        OctMesh mesh;
        std::vector<int32_t> cell, src;  // per new dof: old leaf; per new history point: source
        std::vector<double> xi;          // per new dof: reference coordinates in the old leaf
        std::vector<int32_t> grp_start, grp_idx;  // coarsened parents: old history points to take the min of
    } pending;
    // last gradient forward sweep (checked by the backward sweep)
    struct {
        const void *work = nullptr;
        int n_steps = 0, n_snaps = 0;
        double t0 = 0, dt = 0;
        const double *cur = nullptr;  // executor state after the forward sweep
        double *next = nullptr;
        bool valid = false;
        // every problem parameter the reversal reads (material, laser and track
        // powers, boundary, probes), as seen by the forward sweep
        std::vector<double> problem;
    } grad;
    Law<double> h_law64{}, h_lin64{}, h_zero64{};
    Law<float> h_law32{};
    // implicit-step preconditioner: 0 Jacobi, 1 geometric multigrid V-cycle
    // (boxes: Q1 on the same mesh below Q2, then 2x coarser Q1 meshes)
    int precond = 0, mg_smooth = 2, mg_coarse = 8;
    int newton_forcing = 0;        // 0: every Newton system to lin_rtol; 1: Eisenstat-Walker forcing
    std::vector<pbf_ctx *> mg;     // coarse levels (owned)
    double *d_mg[4] = {};          // fine-level smoother vectors and the V-cycle's input
    std::vector<double> mg_lmax;   // lambda_max(D^-1 A) per level (0 = fine)
    // the V-cycle of the current step as a HIP graph (its kernels and their
    // arguments are fixed within a step), captured on a library stream
    hipStream_t mg_cap = nullptr;
    hipGraphExec_t mg_exec = nullptr;
    double *mg_exec_out = nullptr;
    // kernel timing: 4 events per timed step (cell kernel start/stop, face kernel
    // start/stop), on every `timing_every`-th explicit step
    std::vector<hipEvent_t> tev;
    hipEvent_t ev_read = nullptr;  // completion of a small device-to-host read (Krylov loops)
    double *h_read = nullptr;      // pinned host scalars of that read
    size_t tev_used = 0;
    bool timing = false;
    int timing_every = 1;
    long long timing_seen = 0;
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
long long n_dofs(const pbf_ctx *c)
{
    return c->octree ? c->oct.n_dofs : nodes1(c, 0) * nodes1(c, 1) * nodes1(c, 2);
}
long long n_cells(const pbf_ctx *c) { return c->octree ? c->oct.n_cells : (long long)c->nx * c->ny * c->nz; }
int nq1(const pbf_ctx *c) { return c->degree + 1; }
long long n_hist_cells(const pbf_ctx *c)
{
    if (c->growing) return (long long)c->nx * c->ny * c->nz_full;  // every layer may start as powder
    return c->octree ? c->oct.n_hist_cells : (long long)c->nx * c->ny * c->hist_layers;
}
// sizes of the state arrays and workspace: the whole box when it grows
long long alloc_dofs(const pbf_ctx *c)
{
    if (!c->growing) return n_dofs(c);
    return nodes1(c, 0) * nodes1(c, 1) * ((long long)c->degree * c->nz_full + 1);
}
long long alloc_cells(const pbf_ctx *c)
{
    return c->growing ? (long long)c->nx * c->ny * c->nz_full : n_cells(c);
}
long long n_hist_qp(const pbf_ctx *c)
{
    const long long q = nq1(c);
    return n_hist_cells(c) * q * q * q;
}
int ceil_div(int a, int b) { return (a + b - 1) / b; }
size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

constexpr int kMaxProbes = 4096;

double gauss_point(int degree, int i)
{
    return degree == 1 ? Tables<1>::gp(i) : Tables<2>::gp(i);
}

// history layers: top cell layers that hold a Gauss level within powder_depth of the top
void compute_history_layers(pbf_ctx *c)
{
    c->hist_layers = 0;
    c->powder_levels.clear();
    if (c->octree && c->has_mesh) {
        oct_finish(c->oct, c->dmask, c->has_material ? c->powder_depth : -1.0);
        return;
    }
    if (c->growing) {  // history for every layer (point-major over the whole box, from layer 0)
        c->hist_layers = c->nz;
        return;
    }
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
int segment_length(int nx, int ny, int nz, int ty, int resident_per_cu)
{
    const long long cols = (long long)ceil_div(nx, kTX) * ceil_div(ny, ty);
    const long long slots = 256LL * resident_per_cu;
    const int smin = ceil_div(nz, kMaxSeg);  // at most kMaxSeg segments
    int best = std::max(std::min(nz, 32), smin);
    long long best_cost = -1;
    for (int S = best; S >= smin; --S) {
        const long long blocks = cols * ceil_div(nz, S);
        const long long cost = ((blocks + slots - 1) / slots) * S;
        if (best_cost < 0 || cost < best_cost) {
            best_cost = cost;
            best = S;
        }
    }
    return best;
}

// Boundaries of MZ = ceil(nz / S) z-segments.  Uniform: S layers each (the
// top one takes the remainder).  top_short: the top segment takes S/2 layers
// and the lower ones share the rest evenly (longer ones at the bottom).  The
// top layers of a scan are the costliest (beam, melt pool, powder history),
// and a column's top segment sets the launch time when it is as long as the
// others.
int segment_bounds(int nz, int S, bool top_short, int *zb)
{
    const int MZ = ceil_div(nz, S);
    zb[0] = 0;
    if (!top_short || MZ < 2 || S < 2) {
        for (int s = 1; s <= MZ; ++s) zb[s] = std::min(s * S, nz);
        return MZ;
    }
    const int lower = MZ - 1, rest = nz - S / 2;  // rest >= lower: nz > (MZ - 1) S
    for (int s = 0; s < lower; ++s) zb[s + 1] = zb[s] + rest / lower + (s < rest % lower ? 1 : 0);
    zb[MZ] = nz;
    return MZ;
}

// Column geometry of a cell kernel with columns of 16 x ty cells and the given
// number of resident workgroups per CU (explicit kernels by default, which
// also shorten the top segment).
HaloParams geometry(const pbf_ctx *c, int ty = -1, int resident = -1)
{
    if (c->octree) {  // dof vectors with per-dof Dirichlet flags
        HaloParams h{};
        h.NX = (int)c->oct.n_dofs;
        h.NY = h.NZ = 1;
        h.T_D = c->T_D;
        h.dflag = c->od.dflag;
        h.nlaw = c->d_law64;
        return h;
    }
    const bool top_short = ty < 0;
    if (ty < 0) {
        ty = column_height();
        resident = resident_columns_per_cu(ty);
    }
    HaloParams h{};
    const int P = c->degree;
    const int S = segment_length(c->nx, c->ny, c->nz, ty, resident);
    h.NX = (int)nodes1(c, 0);
    h.NY = (int)nodes1(c, 1);
    h.NZ = (int)nodes1(c, 2);
    h.SX = P * kTX;
    h.SY = P * ty;
    h.MX = ceil_div(c->nx, kTX);
    h.MY = ceil_div(c->ny, ty);
    h.MZ = segment_bounds(c->nz, S, top_short, h.zb);
    h.GX = (long long)(h.MX - 1) * h.NY * h.NZ;
    h.GY = (long long)h.NX * (h.MY - 1) * h.NZ;
    h.GZ = (long long)h.NX * h.NY * (h.MZ - 1);
    h.fNX = fast_div(h.NX);
    h.fNY = fast_div(h.NY);
    h.fNZ = fast_div(h.NZ);
    h.fSX = fast_div(h.SX);
    h.fSY = fast_div(h.SY);
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

// Resident workgroups per CU assumed by the Picard-operator column geometry.
constexpr int kPicardResident = 3;

FaceMap face_map(const HaloParams &h)
{
    return FaceMap{h.GX, h.GY, h.GX + h.GY + h.GZ};
}

// Column-face nodes of a box of nx x ny x nz cells of degree P under columns of
// 16 x ty cells with the given residency (entries per parity slot).
long long face_nodes(int P, int nx, int ny, int nz, int ty, int resident)
{
    const long long NX = (long long)P * nx + 1, NY = (long long)P * ny + 1, NZ = (long long)P * nz + 1;
    const int S = segment_length(nx, ny, nz, ty, resident);
    return (ceil_div(nx, kTX) - 1) * NY * NZ + NX * (ceil_div(ny, ty) - 1) * NZ +
           NX * NY * (ceil_div(nz, S) - 1);
}

// Entries per parity slot: the largest face-node count of the column kernels
// (explicit, Picard, adjoint) over every box the context can take (every
// active height of a growing box).
long long slot_entries(const pbf_ctx *c)
{
    if (c->octree) return 0;
    const int tys[3] = {column_height(), picard_column_height(), adjoint_column_height()};
    const int res[3] = {resident_columns_per_cu(column_height()), kPicardResident,
                         adjoint_resident_columns_per_cu()};
    long long m = 1;
    const int z1 = c->growing ? c->nz_full : c->nz;
    for (int nz = c->growing ? 1 : c->nz; nz <= z1; ++nz)
        for (int g = 0; g < 3; ++g) m = std::max(m, face_nodes(c->degree, c->nx, c->ny, nz, tys[g], res[g]));
    return m;
}

HaloParams adjoint_geometry(const pbf_ctx *c)
{
    return geometry(c, adjoint_column_height(), adjoint_resident_columns_per_cu());
}

long long adjoint_tiles(const pbf_ctx *c)
{
    const HaloParams h = adjoint_geometry(c);
    return (long long)h.MX * h.MY * h.MZ;
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
    std::copy(h.zb, h.zb + h.MZ + 1, p.zb);
    p.hist_cz0 = history ? c->nz - c->hist_layers : c->nz;
    p.hist_write = 1;
    p.n_hist_cells = (int)n_hist_cells(c);
    p.hx = c->L[0] / c->nx;
    p.hy = c->L[1] / c->ny;
    p.hz = c->L[2] / c->nz;
    p.Lz = c->L[2];
    p.detJ = R(p.hx * p.hy * p.hz);
    p.ih2x = R(1.0 / (p.hx * p.hx));
    p.ih2y = R(1.0 / (p.hy * p.hy));
    p.ih2z = R(1.0 / (p.hz * p.hz));
    p.iso = p.ih2x == p.ih2y && p.ih2y == p.ih2z;
    p.ihx = 1.0 / p.hx;
    p.ihy = 1.0 / p.hy;
    p.ihz = 1.0 / p.hz;
    p.T_D = c->T_D;
    p.Tref = std::is_same<R, double>::value ? 0.0 : c->Tref;
    p.dmask = c->dmask;
    p.slots = c->d_slots;
    p.fm = face_map(h);
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

pbf_status oct_upload(pbf_ctx *c, hipStream_t s, bool all);

pbf_status upload_laws(pbf_ctx *c, hipStream_t s)
{
    if (c->octree && c->oct_flags_dirty) {  // Dirichlet flags and history leaves
        pbf_status st = oct_upload(c, s, false);
        if (st) return st;
    }
    if (!c->laws_dirty) return PBF_OK;
    build_law<double>(c, 0.0, false, 0, c->h_law64);
    build_law<float>(c, c->Tref, false, 0, c->h_law32);
    build_law<double>(c, 0.0, true, critical_breakpoint(c), c->h_lin64);
    c->h_zero64 = c->h_lin64;  // k = 0: the operator reduces to the source terms
    c->h_zero64.k0 = 0.0;
    PBF_HIP(c, hipMemcpyAsync(c->d_law64, &c->h_law64, sizeof(Law<double>), hipMemcpyHostToDevice, s));
    PBF_HIP(c, hipMemcpyAsync(c->d_law32, &c->h_law32, sizeof(Law<float>), hipMemcpyHostToDevice, s));
    PBF_HIP(c, hipMemcpyAsync(c->d_lin64, &c->h_lin64, sizeof(Law<double>), hipMemcpyHostToDevice, s));
    PBF_HIP(c, hipMemcpyAsync(c->d_zero64, &c->h_zero64, sizeof(Law<double>), hipMemcpyHostToDevice, s));
    PBF_HIP(c, hipStreamSynchronize(s));
    c->laws_dirty = false;
    return PBF_OK;
}

// law of an operator pass: the material law, the linear law at the critical
// breakpoint (stability estimate: no source, no surface losses), k = 0 (source
// and surface terms only), or k = 0 without the source (surface losses alone)
enum { LAW_FULL = 0, LAW_CRITICAL = 1, LAW_SOURCE = 2, LAW_SURFACE = 3 };

// surface-loss parameters of a pass (off for the stability estimate)
SurfaceLoss surface_params(const pbf_ctx *c, int law)
{
    SurfaceLoss r = c->re;
    if (law == LAW_CRITICAL) r.on = 0;
    r.law = c->d_law64;
    return r;
}

OctParams oct_params(const pbf_ctx *c, const Law<double> *law, const Beam &bm)
{
    OctParams p{};
    p.m = c->od;
    p.law = law;
    p.laser_kind = c->laser_kind;
    p.h_powder = c->h_powder;
    p.two_over_R2 = c->radius > 0 ? 2.0 / (c->radius * c->radius) : 0.0;
    if (bm.on) {
        const double PI = 3.14159265358979323846, R2 = c->radius * c->radius;
        p.laser_on = 1;
        p.xb = bm.xb;
        p.yb = bm.yb;
        p.src_amp = c->laser_kind == 1 ? 2.0 * bm.W / (PI * R2 * c->h_powder) : 2.0 * bm.W / (PI * R2);
    }
    return p;
}

// operator pass on an octree: cell pass into the element buffer, node pass
pbf_status oct_pass(pbf_ctx *c, int mode, int law, const double *Tin, double *Tout, double *f, double *C,
                    double *rc, double t, double dt, hipStream_t s, bool hist_write)
{
    const Law<double> *L = law == LAW_FULL ? c->d_law64 : (law == LAW_CRITICAL ? c->d_lin64 : c->d_zero64);
    const Beam off{false, 0, 0, 0, -1};
    OctParams p = oct_params(c, L, (law == LAW_CRITICAL || law == LAW_SURFACE) ? off : beam_at(c, t));
    p.re = surface_params(c, law);
    p.Tin = Tin;
    p.hist = rc;
    p.has_hist = law == LAW_FULL && rc != nullptr;
    p.hist_write = hist_write ? 1 : 0;
    const bool timed = c->timing && mode == 0 && (c->timing_seen++ % c->timing_every) == 0 &&
                       c->tev_used + 4 <= c->tev.size();
    if (timed) PBF_HIP(c, hipEventRecord(c->tev[c->tev_used], s));
    PBF_HIP(c, launch_oct_cells(c->degree, p, s));
    if (timed) {
        PBF_HIP(c, hipEventRecord(c->tev[c->tev_used + 1], s));
        PBF_HIP(c, hipEventRecord(c->tev[c->tev_used + 2], s));
    }
    OctNodeParams np{};
    np.m = c->od;
    np.Tin = Tin;
    np.Tout = Tout;
    np.fout = f;
    np.Cout = C;
    np.dt = dt;
    np.T_D = c->T_D;
    np.nlaw = law == LAW_CRITICAL ? c->d_lin64 : c->d_law64;
    PBF_HIP(c, launch_oct_nodes(mode, np, s));
    if (timed) {
        PBF_HIP(c, hipEventRecord(c->tev[c->tev_used + 3], s));
        c->tev_used += 4;
    }
    return PBF_OK;
}

// one operator pass: MODE 0 explicit step Tin -> Tout, MODE 1 assemble into f, C
pbf_status operator_pass(pbf_ctx *c, int mode, int precision, int law, const double *Tin,
                         double *Tout, double *f, double *C, double *rc, double t, double dt,
                         hipStream_t s, bool hist_write = true)
{
    if (c->octree) return oct_pass(c, mode, law, Tin, Tout, f, C, rc, t, dt, s, hist_write);
    const bool linear = law == LAW_CRITICAL;
    CellParams<double> pd{};
    CellParams<float> pf{};
    if (precision == PBF_PREC_FP64) {
        pd = cell_params<double>(c, law == LAW_FULL ? c->d_law64 : (linear ? c->d_lin64 : c->d_zero64),
                                 law == LAW_FULL);
        pd.Tin = Tin;
        pd.Tout = Tout;
        pd.fout = f;
        pd.Cout = C;
        pd.hist = rc;
        pd.dt = dt;
        pd.dtr = dt / (linear ? c->h_lin64.rho : c->h_law64.rho);
        pd.hist_write = hist_write ? 1 : 0;
        if (!linear && law != LAW_SURFACE) set_beam(c, pd, t);
        pd.re = surface_params(c, law);
    } else {
        pf = cell_params<float>(c, c->d_law32, true);
        pf.Tin = Tin;
        pf.Tout = Tout;
        pf.fout = f;
        pf.Cout = C;
        pf.hist = rc;
        pf.dt = dt;
        pf.dtr = dt / c->h_law64.rho;
        pf.hist_write = hist_write ? 1 : 0;
        set_beam(c, pf, t);
        pf.re = surface_params(c, law);
    }
    if (linear) pd.nlaw = c->d_lin64;
    const bool timed = c->timing && mode != 1 && (c->timing_seen++ % c->timing_every) == 0 &&
                       c->tev_used + 4 <= c->tev.size();
    hipEvent_t *ev = timed ? &c->tev[c->tev_used] : nullptr;
    PBF_HIP(c, launch_cells(c->degree, precision, mode, column_height(), pd, pf, s, ev ? ev[0] : nullptr,
                            ev ? ev[1] : nullptr));
    HaloParams h = geometry(c);
    if (linear) h.nlaw = c->d_lin64;
    h.Tin = Tin;
    h.Tout = Tout;
    h.fout = f;
    h.Cout = C;
    h.dt = dt;
    const bool faces = h.GX + h.GY + h.GZ > 0;
    PBF_HIP(c, launch_halo(mode, h, s, ev ? ev[2] : nullptr, ev ? ev[3] : nullptr));
    if (timed) {
        if (!faces) {  // no tile-face kernel: zero-length face interval
            PBF_HIP(c, hipEventRecord(ev[2], s));
            PBF_HIP(c, hipEventRecord(ev[3], s));
        }
        c->tev_used += 4;
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
    q.fm = face_map(h);
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
    std::copy(h.zb, h.zb + h.MZ + 1, q.zb);
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

// Picard operator pass (mode 0 apply into y, 1 diagonal into y) on boxes or octrees
pbf_status picard_pass(pbf_ctx *c, int mode, const HaloParams &hp, const double *Tc, const double *Tk,
                       const double *x1, const double *x2, double *y, const double *rc, double dt,
                       const Beam *src, hipStream_t s)
{
    if (!c->octree) {
        const PicardParams q = picard_params(c, hp, Tc, Tk, x1, x2, y, rc, dt, src);
        PBF_HIP(c, launch_picard(c->degree, mode, q, hp, s));
        return PBF_OK;
    }
    const Beam off{false, 0, 0, 0, -1};
    OctParams p = oct_params(c, c->d_law64, (src && mode == 0) ? *src : off);
    p.Tc = Tc;
    p.Tk = Tk;
    p.x1 = x1;
    p.x2 = x2;
    p.hist = const_cast<double *>(rc);
    p.has_hist = rc != nullptr;
    p.inv_dt = 1.0 / dt;
    PBF_HIP(c, launch_oct_picard(c->degree, mode, p, s));
    OctNodeParams np{};
    np.m = c->od;
    np.Tout = y;
    PBF_HIP(c, launch_oct_nodes(mode == 0 ? 2 : 3, np, s));
    return PBF_OK;
}

// ---- probes and adjoint ------------------------------------------------------

ProbeSet probe_set(const pbf_ctx *c)
{
    ProbeSet ps{};
    ps.cell = c->d_probe_cell;
    ps.xi = c->d_probe_xi;
    ps.target = c->d_probe_target;
    ps.n = (int)c->probe_target.size();
    ps.P = c->degree;
    ps.NX = (int)nodes1(c, 0);
    ps.NY = (int)nodes1(c, 1);
    ps.NXY = (long long)ps.NX * ps.NY;
    return ps;
}

pbf_status upload_probes(pbf_ctx *c, hipStream_t s)
{
    if (!c->probes_dirty) return PBF_OK;
    const size_t n = c->probe_target.size();
    if (n > 0) {
        PBF_HIP(c, hipMemcpyAsync(c->d_probe_cell, c->probe_cell.data(), 3 * n * sizeof(int),
                                  hipMemcpyHostToDevice, s));
        PBF_HIP(c, hipMemcpyAsync(c->d_probe_xi, c->probe_xi.data(), 3 * n * sizeof(double),
                                  hipMemcpyHostToDevice, s));
        PBF_HIP(c, hipMemcpyAsync(c->d_probe_target, c->probe_target.data(), n * sizeof(double),
                                  hipMemcpyHostToDevice, s));
        PBF_HIP(c, hipStreamSynchronize(s));
    }
    c->probes_dirty = false;
    return PBF_OK;
}

AdjointParams adjoint_params(const pbf_ctx *c, const HaloParams &h, const double *T, const double *Tn1,
                             const double *rc, const double *lam_next, double *lam, double *mu, double dt,
                             const Beam &bm)
{
    AdjointParams a{};
    a.T = T;
    a.Tn1 = Tn1;
    a.lam = lam_next;
    a.lam_out = lam;
    a.hist = rc;
    a.mu = mu;
    a.slots = c->d_slots;
    a.fm = face_map(h);
    a.partials = c->d_tiles;
    a.nx = c->nx;
    a.ny = c->ny;
    a.nz = c->nz;
    a.NX = h.NX;
    a.NY = h.NY;
    a.NZ = h.NZ;
    a.MX = h.MX;
    a.MY = h.MY;
    a.MZ = h.MZ;
    a.ntiles = h.MX * h.MY * h.MZ;
    a.tiles_per_xcd = ceil_div(a.ntiles, 8);
    std::copy(h.zb, h.zb + h.MZ + 1, a.zb);
    a.hist_cz0 = c->nz - c->hist_layers;
    a.n_hist_cells = (int)n_hist_cells(c);
    a.hx = c->L[0] / c->nx;
    a.hy = c->L[1] / c->ny;
    a.hz = c->L[2] / c->nz;
    a.Lz = c->L[2];
    a.detJ = a.hx * a.hy * a.hz;
    a.ih2x = 1.0 / (a.hx * a.hx);
    a.ih2y = 1.0 / (a.hy * a.hy);
    a.ih2z = 1.0 / (a.hz * a.hz);
    a.dt = dt;
    a.dmask = c->dmask;
    a.laser_kind = c->laser_kind;
    const double depth_cells = (c->L[2] - c->h_powder) / a.hz;
    a.src_cz0 = std::max(0, (int)std::floor(depth_cells) - 1);
    a.h_powder = c->h_powder;
    a.two_over_R2 = c->radius > 0 ? 2.0 / (c->radius * c->radius) : 0.0;
    a.src_on = bm.on ? 1 : 0;
    if (bm.on) {
        const double PI = 3.14159265358979323846, R2 = c->radius * c->radius;
        a.xb = bm.xb;
        a.yb = bm.yb;
        a.src_unit = c->laser_kind == 1 ? 2.0 / (PI * R2 * c->h_powder) : 2.0 / (PI * R2);
    }
    a.law = c->d_law64;
    return a;
}

// one reverse step at state (T = T_n, rc = r^{n-1}), time t, with Tn1 = T_{n+1}
pbf_status adjoint_step(pbf_ctx *c, const double *T, const double *Tn1, const double *rc, const double *lam_next,
                        double *lam, double *mu, double t, double dt, double *dJdW, hipStream_t s)
{
    const Beam bm = beam_at(c, t);
    AdjointHalo ah{};
    ah.h = adjoint_geometry(c);
    ah.h.Tin = T;
    ah.h.dt = dt;
    ah.Tn1 = Tn1;
    ah.lam = lam_next;
    ah.lam_out = lam;
    const AdjointParams ap = adjoint_params(c, ah.h, T, Tn1, rc, lam_next, lam, mu, dt, bm);
    PBF_HIP(c, launch_adjoint(c->degree, ap, ah, s));
    if (bm.on) PBF_HIP(c, launch_adjoint_finish(c->d_tiles, ap.ntiles, dJdW, bm.track, s));
    return PBF_OK;
}

// device buffer of the checkpointed gradient: snapshots, three rotating
// temperature buffers, history, adjoint vectors, parameter gradients
struct GradWork {
    double *snapT, *snapR, *B[3], *rcur, *rtmp, *lam, *lam2, *mu, *dJdW, *powers, *J;
    size_t bytes;
};

GradWork grad_layout(const pbf_ctx *c, int n_snaps, char *base)
{
    const size_t N = (size_t)n_dofs(c), H = (size_t)std::max(n_hist_qp(c), 1LL),
                 K = std::max<size_t>(c->tracks.size(), 1);
    GradWork w{};
    size_t off = 0;
    auto take = [&](size_t n) {
        double *p = base ? (double *)(base + off) : nullptr;
        off += align256(n * sizeof(double));
        return p;
    };
    w.snapT = take((size_t)n_snaps * N);
    w.snapR = take((size_t)n_snaps * H);
    for (int k = 0; k < 3; ++k) w.B[k] = take(N);
    w.rcur = take(H);
    w.rtmp = take(H);
    w.lam = take(N);
    w.lam2 = take(N);
    w.mu = take(H);
    w.dJdW = take(K);
    w.powers = take(K);
    w.J = take(1);
    w.bytes = off;
    return w;
}

// Executor state: the temperature of the current state (a work buffer or a
// snapshot, read only) and T_{n+1} of the next reverse step (a work buffer).
// Advances ping-pong between the buffers that hold neither; an advance that
// ends in a snapshot writes its last step there; a restore only points at the
// snapshot (the history, updated in place by steps, is copied).
struct GradState {
    const double *cur = nullptr;
    double *next = nullptr;
    int step = 0;
};

double *free_buffer(const GradWork &w, const GradState &g)
{
    for (double *b : w.B)
        if (b != g.cur && b != g.next) return b;
    return nullptr;
}

// execute schedule actions [i0, i1); TURN actions run adjoint steps
pbf_status run_actions(pbf_ctx *c, const std::vector<pbf_revolve_action> &acts, size_t i0, size_t i1,
                       const GradWork &w, GradState &g, double *&lam, double *&lam2, double t0, double dt,
                       hipStream_t s)
{
    const size_t N = (size_t)n_dofs(c), H = (size_t)n_hist_qp(c);
    auto slotT = [&](int k) { return w.snapT + (size_t)k * N; };
    for (size_t i = i0; i < i1; ++i) {
        const pbf_revolve_action &a = acts[i];
        if (a.kind == PBF_ACT_ADVANCE) {
            const bool into_slot = i + 1 < i1 && acts[i + 1].kind == PBF_ACT_STORE && acts[i + 1].step == a.step;
            for (int n = g.step; n < a.step; ++n) {
                double *dst = (n == a.step - 1 && into_slot) ? slotT(acts[i + 1].slot) : free_buffer(w, g);
                pbf_status st = operator_pass(c, 0, PBF_PREC_FP64, LAW_FULL, g.cur, dst, nullptr, nullptr,
                                              H ? w.rcur : nullptr, t0 + n * dt, dt, s);
                if (st) return st;
                g.cur = dst;
            }
            g.step = a.step;
        } else if (a.kind == PBF_ACT_STORE) {
            if (g.step != a.step) return fail(c, PBF_ESTATE, "checkpoint schedule out of step");
            if (g.cur != slotT(a.slot))
                PBF_HIP(c, hipMemcpyAsync(slotT(a.slot), g.cur, N * sizeof(double), hipMemcpyDeviceToDevice, s));
            if (H) PBF_HIP(c, hipMemcpyAsync(w.snapR + (size_t)a.slot * H, w.rcur, H * sizeof(double),
                                             hipMemcpyDeviceToDevice, s));
        } else if (a.kind == PBF_ACT_RESTORE) {
            g.cur = slotT(a.slot);
            if (H) PBF_HIP(c, hipMemcpyAsync(w.rcur, w.snapR + (size_t)a.slot * H, H * sizeof(double),
                                             hipMemcpyDeviceToDevice, s));
            g.step = a.step;
        } else if (a.kind == PBF_ACT_TURN) {
            if (g.step != a.step || !g.next)
                return fail(c, PBF_ESTATE, "checkpoint schedule out of step (%d vs %d)", g.step, a.step);
            pbf_status st = adjoint_step(c, g.cur, g.next, H ? w.rcur : nullptr, lam, lam2, H ? w.mu : nullptr,
                                         t0 + a.step * dt, dt, w.dJdW, s);
            if (st) return st;
            std::swap(lam, lam2);
            // T_n is T_{n+1} of the next reverse step; keep it in a work buffer
            double *keep = nullptr;
            for (double *b : w.B)
                if (b == g.cur) keep = b;
            if (!keep) {
                keep = g.next;  // T_{n+1} is no longer needed
                PBF_HIP(c, hipMemcpyAsync(keep, g.cur, N * sizeof(double), hipMemcpyDeviceToDevice, s));
            }
            g.next = keep;
        }
    }
    return PBF_OK;
}

// octree tables in the workspace: the bytes they take and, when base is not
// NULL, the device view carved from base into c->od (sizing leaves c untouched)
size_t oct_tables(pbf_ctx *c, char *base)
{
    if (!c->octree) return 0;
    const OctMesh &m = c->oct;
    const int NN = nq1(c) * nq1(c) * nq1(c);
    size_t off = 0;
    auto take = [&](size_t n) {
        char *p = base ? base + off : nullptr;
        off += align256(n);
        return p;
    };
    OctDev tmp{};
    OctDev &d = base ? c->od : tmp;
    d.cidx = (const int32_t *)take(m.cidx.size() * 4);
    d.hstart = (const int32_t *)take(m.hstart.size() * 4);
    d.hdof = (const int32_t *)take(m.hdof.size() * 4);
    d.hw = (const double *)take(m.hw.size() * 8);
    d.leaf = (const int32_t *)take(m.leaf.size() * 4);
    d.cell_hist = (const int32_t *)take((size_t)m.n_cells * 4);
    d.nstart = (const int32_t *)take(m.nstart.size() * 4);
    d.nslot = (const int32_t *)take(m.nslot.size() * 4);
    d.nw = m.nw_f32 ? nullptr : (const double *)take(m.nw.size() * 8);
    d.nwf = m.nw_f32 ? (const float *)take(m.nwf.size() * 4) : nullptr;
    d.nw_f32 = m.nw_f32 ? 1 : 0;
    d.mass = (const double *)take(m.mass.size() * 8);
    d.dflag = (const unsigned char *)take((size_t)m.n_dofs);
    d.hist_z = (const double *)take(std::max<size_t>(m.hist_z.size(), 2) * 8);
    d.E = (double *)take((size_t)NN * m.n_cells * 8);
    d.n_cells = (int)m.n_cells;
    d.n_dofs = (int)m.n_dofs;
    d.n_hist_cells = (int)m.n_hist_cells;
    d.maxl = m.maxl;
    d.top_iz = (int)m.top;
    d.ux = m.unit[0];
    d.uy = m.unit[1];
    d.uz = m.unit[2];
    d.Lz = (double)m.top * m.unit[2];
    return off;
}

pbf_status oct_upload(pbf_ctx *c, hipStream_t s, bool all)
{
    const OctMesh &m = c->oct;
    const OctDev &d = c->od;
    auto put = [&](const void *dst, const void *src, size_t n) -> hipError_t {
        return n ? hipMemcpyAsync(const_cast<void *>(dst), src, n, hipMemcpyHostToDevice, s) : hipSuccess;
    };
    c->oct_flags_dirty = false;
    if (!all) {
        PBF_HIP(c, put(d.dflag, m.dflag.data(), m.dflag.size()));
        PBF_HIP(c, put(d.cell_hist, m.cell_hist.data(), m.cell_hist.size() * 4));
        PBF_HIP(c, put(d.hist_z, m.hist_z.data(), m.hist_z.size() * 8));
        PBF_HIP(c, hipStreamSynchronize(s));
        return PBF_OK;
    }
    PBF_HIP(c, put(d.cidx, m.cidx.data(), m.cidx.size() * 4));
    PBF_HIP(c, put(d.hstart, m.hstart.data(), m.hstart.size() * 4));
    PBF_HIP(c, put(d.hdof, m.hdof.data(), m.hdof.size() * 4));
    PBF_HIP(c, put(d.hw, m.hw.data(), m.hw.size() * 8));
    PBF_HIP(c, put(d.leaf, m.leaf.data(), m.leaf.size() * 4));
    PBF_HIP(c, put(d.cell_hist, m.cell_hist.data(), m.cell_hist.size() * 4));
    PBF_HIP(c, put(d.nstart, m.nstart.data(), m.nstart.size() * 4));
    PBF_HIP(c, put(d.nslot, m.nslot.data(), m.nslot.size() * 4));
    if (m.nw_f32) PBF_HIP(c, put(d.nwf, m.nwf.data(), m.nwf.size() * 4));
    else PBF_HIP(c, put(d.nw, m.nw.data(), m.nw.size() * 8));
    PBF_HIP(c, put(d.mass, m.mass.data(), m.mass.size() * 8));
    PBF_HIP(c, put(d.dflag, m.dflag.data(), m.dflag.size()));
    PBF_HIP(c, put(d.hist_z, m.hist_z.data(), m.hist_z.size() * 8));
    PBF_HIP(c, hipStreamSynchronize(s));
    return PBF_OK;
}

}  // namespace

// ---- geometric multigrid preconditioner of the implicit systems (boxes) ----
// Levels: the fine problem (Q2 or Q1), Q1 on the same mesh when the fine
// degree is 2, then Q1 on meshes coarsened 2x in every direction while all
// cell counts are even and the coarse lattice keeps more than kMgCoarseNodes
// nodes.  Every level rediscretizes the Picard matrix C(T_n)/dt + K(T^i) with
// the temperatures injected from the next finer level (coarse nodes are fine
// nodes) and the consolidated fraction taken as 1 (the coarse levels carry no
// powder history: only the preconditioner changes, not the solution).  The
// V-cycle smooths with Chebyshev polynomials of D^-1 A (the same polynomial
// before and after the coarse correction, so the cycle is symmetric and
// positive definite and serves CG), restricts with the transpose of trilinear
// interpolation, and treats the coarsest level with a higher-degree Chebyshev
// polynomial.
namespace {
constexpr long long kMgCoarseNodes = 4096;
constexpr double kMgRange = 15.0, kMgCoarseRange = 60.0, kMgSafety = 1.15;

struct MgLevel {
    pbf_ctx *c;
    long long N;
    HaloParams ge, hp;
    const double *Tn;
    double *Ti, *diag, *x, *b, *r, *d, *t;
    const double *coef;
    bool fine;
};

pbf_status mg_build_levels(pbf_ctx *c)
{
    for (pbf_ctx *l : c->mg) pbf_destroy(l);
    c->mg.clear();
    int deg = c->degree, nx = c->nx, ny = c->ny, nz = c->nz;
    auto nodes = [](int d, int a, int b, int e) { return (long long)(d * a + 1) * (d * b + 1) * (d * e + 1); };
    for (;;) {
        int nd = 1, ax = nx, ay = ny, az = nz;
        if (deg == 1) {
            if (nx % 2 || ny % 2 || nz % 2) break;
            ax = nx / 2;
            ay = ny / 2;
            az = nz / 2;
        }
        if (deg == 1 && nodes(1, ax, ay, az) <= kMgCoarseNodes / 8) break;
        if (deg == 1 && nodes(1, nx, ny, nz) <= kMgCoarseNodes) break;
        pbf_ctx *l = nullptr;
        if (pbf_create(&l) != PBF_OK) return fail(c, PBF_ENOMEM, "multigrid level");
        c->mg.push_back(l);
        pbf_status st = pbf_mesh_box(l, nd, ax, ay, az, c->L[0], c->L[1], c->L[2]);
        if (!st) st = pbf_set_dirichlet(l, c->dmask, c->T_D);
        if (!st) {
            pbf_material m{};
            m.n_bp = c->n_bp;
            m.T_bp = c->T_bp;
            m.k_bp = c->k_bp;
            m.cp_bp = c->cp_bp;
            m.rho = c->rho;
            m.T_s = c->T_s;
            m.T_l = c->T_l;
            m.latent = c->latent;
            m.powder_k_factor = c->phi;
            m.powder_depth = 0.0;  // no history on coarse levels
            st = pbf_set_material(l, &m);
        }
        if (st) return fail(c, st, "multigrid level: %s", l->err.c_str());
        deg = 1;
        nx = ax;
        ny = ay;
        nz = az;
    }
    c->mg_lmax.assign(c->mg.size() + 1, 0.0);
    return PBF_OK;
}

// the levels of the current solve; level 0 solves with the fine operator's cache
std::vector<MgLevel> mg_levels(pbf_ctx *c, const double *T_n, double *Ti, double *diag, const double *fine_coef)
{
    std::vector<MgLevel> L;
    MgLevel f{};
    f.c = c;
    f.N = n_dofs(c);
    f.ge = geometry(c);
    f.hp = geometry(c, picard_column_height(), kPicardResident);
    f.Tn = T_n;
    f.Ti = Ti;
    f.diag = diag;
    f.r = c->d_mg[0];
    f.d = c->d_mg[1];
    f.t = c->d_mg[2];
    f.coef = fine_coef;
    f.fine = true;
    L.push_back(f);
    for (pbf_ctx *l : c->mg) {
        MgLevel v{};
        v.c = l;
        v.N = n_dofs(l);
        v.ge = geometry(l);
        v.hp = geometry(l, picard_column_height(), kPicardResident);
        v.Tn = l->d_cg[0];
        v.Ti = l->d_cg[1];
        v.diag = l->d_cg[2];
        v.x = l->d_cg[3];
        v.b = l->d_cg[4];
        v.r = l->d_cg[5];
        v.d = l->d_cg[6];
        v.t = l->d_cg[7];
        v.coef = l->d_coef;
        v.fine = false;
        L.push_back(v);
    }
    return L;
}

// y = A_l x (Picard matrix of the level, from its coefficient cache)
pbf_status mg_apply(const MgLevel &v, const double *x, double *y, double dt, hipStream_t s)
{
    pbf_ctx *c = v.c;
    PicardParams pa = picard_params(c, v.ge, v.Tn, v.Ti, x, x, y, nullptr, dt, nullptr);
    pa.coef = const_cast<double *>(v.coef);
    pa.ncells = (long long)c->nx * c->ny * c->nz;
    PBF_HIP(c, launch_picard_capply(c->degree, false, pa, v.ge, s));
    return PBF_OK;
}

// coarse-level temperatures, diagonals and coefficient caches for T^i
pbf_status mg_setup(pbf_ctx *c, std::vector<MgLevel> &L, double dt, hipStream_t s)
{
    for (size_t l = 1; l < L.size(); ++l) {
        MgLevel &v = L[l];
        const MgLevel &f = L[l - 1];
        PBF_HIP(c, launch_mg_inject(const_cast<double *>(v.Tn), f.Tn, v.ge, f.ge.NX, f.ge.NY, s));
        PBF_HIP(c, launch_mg_inject(v.Ti, f.Ti, v.ge, f.ge.NX, f.ge.NY, s));
        pbf_status st = picard_pass(v.c, 1, v.hp, v.Tn, v.Ti, nullptr, nullptr, v.diag, nullptr, dt, nullptr, s);
        if (st) return fail(c, st, "multigrid level: %s", v.c->err.c_str());
        PicardParams pc = picard_params(v.c, v.ge, v.Tn, v.Ti, nullptr, nullptr, nullptr, nullptr, dt, nullptr);
        pc.coef = const_cast<double *>(v.coef);
        pc.ncells = (long long)v.c->nx * v.c->ny * v.c->nz;
        PBF_HIP(c, launch_picard_coef(1, false, pc, s));
    }
    return PBF_OK;
}

// forget the captured V-cycle (new eigenvalue bounds, step or buffers)
void mg_graph_reset(pbf_ctx *c)
{
    if (c->mg_exec) (void)hipGraphExecDestroy(c->mg_exec);
    c->mg_exec = nullptr;
    c->mg_exec_out = nullptr;
}

// lambda_max(D^-1 A) of every level by power iteration (synchronizes)
pbf_status mg_eigen(pbf_ctx *c, std::vector<MgLevel> &L, double dt, hipStream_t s)
{
    for (size_t l = 0; l < L.size(); ++l) {
        MgLevel &v = L[l];
        double *vec = v.d, *w = v.t;
        PBF_HIP(c, launch_seed(vec, v.N, s));  // fixed pseudo-random start (all frequencies)
        double lam = 0.0;
        for (int it = 0; it < 12; ++it) {
            pbf_status st = mg_apply(v, vec, w, dt, s);
            if (st) return st;
            PBF_HIP(c, launch_div(w, w, v.diag, v.N, s));
            PBF_HIP(c, launch_dot_to(vec, w, c->d_partials, c->d_scal + SC_MG, v.N, s));
            PBF_HIP(c, launch_dot_to(vec, vec, c->d_partials, c->d_scal + SC_MG + 1, v.N, s));
            PBF_HIP(c, launch_dot_to(w, w, c->d_partials, c->d_scal + SC_MG + 2, v.N, s));
            double h[3];
            PBF_HIP(c, hipMemcpyAsync(h, c->d_scal + SC_MG, sizeof h, hipMemcpyDeviceToHost, s));
            PBF_HIP(c, hipStreamSynchronize(s));
            if (!(h[1] > 0) || !(h[2] > 0)) break;
            lam = h[0] / h[1];
            PBF_HIP(c, launch_div_scalar(vec, w, std::sqrt(h[2]), v.N, s));
        }
        if (!(lam > 0) || !std::isfinite(lam)) return fail(c, PBF_ENONFINITE, "multigrid: no eigenvalue estimate");
        c->mg_lmax[l] = kMgSafety * lam;
    }
    mg_graph_reset(c);
    return PBF_OK;
}

// x <- Chebyshev sweep of `degree` steps on A_l x = b (from x = 0 if zero);
// eigenvalues of D^-1 A in [lmax / range, lmax]
pbf_status mg_smooth(pbf_ctx *c, const MgLevel &v, const double *b, double *x, int degree, double lmax,
                     double range, bool zero, double dt, hipStream_t s)
{
    const double l0 = lmax / range, l1 = lmax;
    const double theta = 0.5 * (l1 + l0), delta = 0.5 * (l1 - l0), sigma = theta / delta;
    double rho = 1.0 / sigma;
    pbf_status st;
    // first step: d = D^-1 r / theta
    if (zero) {
        PBF_HIP(c, launch_cheb(x, v.d, b, v.diag, 0.0, 1.0 / theta, true, v.N, s));
    } else {
        if ((st = mg_apply(v, x, v.t, dt, s))) return st;
        PBF_HIP(c, launch_cheb_res(x, v.d, b, v.t, v.diag, 0.0, 1.0 / theta, v.N, s));
    }
    for (int k = 1; k < degree; ++k) {
        if ((st = mg_apply(v, x, v.t, dt, s))) return st;
        const double rho_new = 1.0 / (2.0 * sigma - rho);
        PBF_HIP(c, launch_cheb_res(x, v.d, b, v.t, v.diag, rho_new * rho, 2.0 * rho_new / delta, v.N, s));
        rho = rho_new;
    }
    return PBF_OK;
}

pbf_status mg_vcycle(pbf_ctx *c, std::vector<MgLevel> &L, const double *r, double *z, double dt, hipStream_t s);

// z = M^-1 r: the input is copied to a fixed buffer and the V-cycle, captured
// once per step as a graph (one launch instead of ~100), replayed on s
pbf_status mg_precond(pbf_ctx *c, std::vector<MgLevel> &L, const double *r, double *z, double dt, hipStream_t s)
{
    const long long N = L[0].N;
    PBF_HIP(c, hipMemcpyAsync(c->d_mg[3], r, N * sizeof(double), hipMemcpyDeviceToDevice, s));
    if (!c->mg_exec || c->mg_exec_out != z) {
        mg_graph_reset(c);
        if (!c->mg_cap) PBF_HIP(c, hipStreamCreateWithFlags(&c->mg_cap, hipStreamNonBlocking));
        PBF_HIP(c, hipStreamBeginCapture(c->mg_cap, hipStreamCaptureModeThreadLocal));
        pbf_status st = mg_vcycle(c, L, c->d_mg[3], z, dt, c->mg_cap);
        hipGraph_t g = nullptr;
        const hipError_t e = hipStreamEndCapture(c->mg_cap, &g);
        if (st) {
            if (g) (void)hipGraphDestroy(g);
            return st;
        }
        if (e != hipSuccess) return fail(c, PBF_EDEVICE, "V-cycle capture: %s", hipGetErrorString(e));
        const hipError_t ei = hipGraphInstantiate(&c->mg_exec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (ei != hipSuccess) {
            c->mg_exec = nullptr;
            return fail(c, PBF_EDEVICE, "V-cycle graph: %s", hipGetErrorString(ei));
        }
        c->mg_exec_out = z;
    }
    PBF_HIP(c, hipGraphLaunch(c->mg_exec, s));
    return PBF_OK;
}

// z = M^-1 r by one V-cycle
pbf_status mg_vcycle(pbf_ctx *c, std::vector<MgLevel> &L, const double *r, double *z, double dt, hipStream_t s)
{
    L[0].b = const_cast<double *>(r);
    L[0].x = z;
    const size_t nl = L.size();
    pbf_status st;
    for (size_t l = 0; l + 1 < nl; ++l) {
        MgLevel &v = L[l];
        if ((st = mg_smooth(c, v, v.b, v.x, c->mg_smooth, c->mg_lmax[l], kMgRange, true, dt, s))) return st;
        if ((st = mg_apply(v, v.x, v.t, dt, s))) return st;
        MgLevel &w = L[l + 1];
        PBF_HIP(c, launch_mg_restrict_res(w.b, v.b, v.t, w.ge, v.ge.NX, v.ge.NY, v.ge.NZ, s));
    }
    MgLevel &cl = L[nl - 1];
    if ((st = mg_smooth(c, cl, cl.b, cl.x, c->mg_coarse, c->mg_lmax[nl - 1], kMgCoarseRange, true, dt, s)))
        return st;
    for (size_t l = nl - 1; l-- > 0;) {
        MgLevel &v = L[l];
        PBF_HIP(c, launch_mg_prolong_add(v.x, L[l + 1].x, v.ge, L[l + 1].ge.NX, L[l + 1].ge.NY, s));
        if ((st = mg_smooth(c, v, v.b, v.x, c->mg_smooth, c->mg_lmax[l], kMgRange, false, dt, s))) return st;
    }
    return PBF_OK;
}
}  // namespace

// ---- explicit steps without a workspace ----------------------------------
// The scratch of the explicit step on boxes (the device copies of the laws and
// the parity slots of the column-face partial sums) lives in one static device
// array per GPU.  Host code never names the array in a launch or a copy: its
// device address is taken once per device with hipGetSymbolAddress (with that
// device current) and kept here.
namespace {
constexpr size_t kStaticScratchBytes = size_t(32) << 20;
__device__ __align__(256) char scratch[kStaticScratchBytes];
constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
char *g_scratch_ptr[kMaxScratchDevices] = {};

// device address of the static scratch array on the current device
pbf_status static_scratch(pbf_ctx *c, char **out)
{
    int dev = -1;
    PBF_HIP(c, hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxScratchDevices)
        return fail(c, PBF_EDEVICE, "device %d: the static scratch supports devices 0..%d", dev,
                    kMaxScratchDevices - 1);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(c, PBF_EDEVICE, "hipGetSymbolAddress of the static scratch on device %d: %s", dev,
                        hipGetErrorString(e));
        g_scratch_ptr[dev] = static_cast<char *>(ptr);
    }
    *out = g_scratch_ptr[dev];
    return PBF_OK;
}

// Points the context's law and slot arrays into the static scratch for the
// duration of one call and restores the bound workspace's pointers after it.
struct ScratchBinding {
    pbf_ctx *c;
    Law<double> *law64, *lin64, *zero64;
    Law<float> *law32;
    double *slots;
    bool laws_dirty;
    ScratchBinding(pbf_ctx *ctx, char *base)
        : c(ctx), law64(ctx->d_law64), lin64(ctx->d_lin64), zero64(ctx->d_zero64), law32(ctx->d_law32),
          slots(ctx->d_slots), laws_dirty(ctx->laws_dirty)
    {
        char *p = base;
        c->d_law64 = (Law<double> *)p;
        p += align256(sizeof(Law<double>));
        c->d_lin64 = (Law<double> *)p;
        p += align256(sizeof(Law<double>));
        c->d_zero64 = (Law<double> *)p;
        p += align256(sizeof(Law<double>));
        c->d_law32 = (Law<float> *)p;
        p += align256(sizeof(Law<float>));
        c->d_slots = (double *)p;
        c->laws_dirty = true;  // another call may have left its own laws in the array
    }
    ~ScratchBinding()
    {
        c->d_law64 = law64;
        c->d_lin64 = lin64;
        c->d_zero64 = zero64;
        c->d_law32 = law32;
        c->d_slots = slots;
        c->laws_dirty = laws_dirty;
    }
};
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
    for (pbf_ctx *l : ctx->mg) pbf_destroy(l);
    if (ctx->mg_exec) (void)hipGraphExecDestroy(ctx->mg_exec);
    if (ctx->mg_cap) (void)hipStreamDestroy(ctx->mg_cap);
    for (hipEvent_t e : ctx->tev) (void)hipEventDestroy(e);
    if (ctx->ev_read) (void)hipEventDestroy(ctx->ev_read);
    if (ctx->h_read) (void)hipHostFree(ctx->h_read);
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
    // the column kernels address the degree+1 node planes of a cell layer with
    // 32-bit offsets
    if (NX * NY * (degree + 1) >= (1LL << 31)) return fail(c, PBF_EMESH, "mesh too large: node planes too big");
    c->has_mesh = true;
    c->octree = false;
    c->oct = OctMesh{};
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

static pbf_status mesh_octree(pbf_ctx *c, int degree, int nx, int ny, int nz, double Lx, double Ly, double Lz,
                              int max_level, int64_t top, bool growing, int64_t n_leaves, const int32_t *leaves)
{
    if (!c) return fail(nullptr, PBF_EINVAL, "pbf_mesh_octree: ctx is NULL");
    if (degree != 1 && degree != 2) return fail(c, PBF_EMESH, "degree %d not supported (1 or 2)", degree);
    if (nx < 1 || ny < 1 || nz < 1) return fail(c, PBF_EINVAL, "coarse cell counts must be >= 1");
    if (!(Lx > 0 && Ly > 0 && Lz > 0)) return fail(c, PBF_EINVAL, "box lengths must be > 0");
    if (!leaves) return fail(c, PBF_EINVAL, "leaves is NULL");
    const int n0[3] = {nx, ny, nz};
    const double L[3] = {Lx, Ly, Lz};
    OctMesh m;
    std::string err;
    if (!oct_build(m, degree, max_level, n0, L, n_leaves, leaves, err, top))
        return fail(c, PBF_EMESH, "%s", err.c_str());
    m.growing = growing;
    c->has_mesh = true;
    c->octree = true;
    c->oct = std::move(m);
    c->degree = degree;
    c->nx = nx;
    c->ny = ny;
    c->nz = nz;
    c->L[0] = Lx;
    c->L[1] = Ly;
    c->L[2] = Lz;
    c->bound = false;
    c->laws_dirty = true;
    c->pending.ready = false;
    compute_history_layers(c);
    return PBF_OK;
}

pbf_status pbf_mesh_octree(pbf_ctx *c, int degree, int nx, int ny, int nz, double Lx, double Ly, double Lz,
                           int max_level, int64_t n_leaves, const int32_t *leaves)
{
    return mesh_octree(c, degree, nx, ny, nz, Lx, Ly, Lz, max_level, -1, false, n_leaves, leaves);
}

pbf_status pbf_mesh_octree_growing(pbf_ctx *c, int degree, int nx, int ny, int nz, double Lx, double Ly, double Lz,
                                   int max_level, int64_t top, int64_t n_leaves, const int32_t *leaves)
{
    if (c && top < 1) return fail(c, PBF_EINVAL, "the active top must be >= 1 finest cell");
    return mesh_octree(c, degree, nx, ny, nz, Lx, Ly, Lz, max_level, top, true, n_leaves, leaves);
}

pbf_status pbf_octree_history_min(pbf_ctx *c, const double *rc, double *rc_min, void *stream)
{
    if (!c) return fail(nullptr, PBF_EINVAL, "ctx is NULL");
    if (!c->octree) return fail(c, PBF_ESTATE, "no octree mesh");
    if (!rc_min) return fail(c, PBF_EINVAL, "rc_min is NULL");
    const OctMesh &m = c->oct;
    std::fill(rc_min, rc_min + m.n_cells, 1.0);
    const int64_t nq = n_hist_qp(c);
    if (nq == 0) return PBF_OK;
    if (!rc) return fail(c, PBF_EINVAL, "rc is NULL but the mesh has history");
    std::vector<double> h(nq);
    hipStream_t s = (hipStream_t)stream;
    PBF_HIP(c, hipMemcpyAsync(h.data(), rc, nq * sizeof(double), hipMemcpyDeviceToHost, s));
    PBF_HIP(c, hipStreamSynchronize(s));
    const int64_t npt = (int64_t)(c->degree + 1) * (c->degree + 1) * (c->degree + 1);
    for (int64_t e = 0; e < m.n_cells; ++e) {
        const int32_t hc = m.cell_hist[e];
        if (hc < 0) continue;
        double v = h[hc];
        for (int64_t q = 1; q < npt; ++q) v = std::min(v, h[q * m.n_hist_cells + hc]);
        rc_min[e] = v;
    }
    return PBF_OK;
}

pbf_status pbf_octree_layer_leaves(pbf_ctx *c, const double *rc_min, int64_t new_top, int64_t d_haz, double r_coarsen,
                                   int32_t *leaves, int64_t capacity, int64_t *n_leaves)
{
    if (!c) return fail(nullptr, PBF_EINVAL, "ctx is NULL");
    if (!n_leaves) return fail(c, PBF_EINVAL, "n_leaves is NULL");
    if (!c->octree || !c->oct.growing) return fail(c, PBF_ESTATE, "no growing octree (pbf_mesh_octree_growing)");
    if (d_haz < 0 || !std::isfinite(r_coarsen)) return fail(c, PBF_EINVAL, "need d_haz >= 0 and a finite r_coarsen");
    const OctMesh &m = c->oct;
    std::vector<double> rmin(m.n_cells, 1.0);
    if (rc_min) std::copy(rc_min, rc_min + m.n_cells, rmin.begin());
    std::vector<int32_t> out;
    std::string err;
    if (!oct_layer_leaves(m, rmin, new_top, d_haz, r_coarsen, out, err)) return fail(c, PBF_EINVAL, "%s", err.c_str());
    *n_leaves = (int64_t)(out.size() / 4);
    if (!leaves) return PBF_OK;
    if (capacity < *n_leaves)
        return fail(c, PBF_ENOMEM, "leaf array holds %lld leaves, %lld needed", (long long)capacity, (long long)*n_leaves);
    std::copy(out.begin(), out.end(), leaves);
    return PBF_OK;
}

pbf_status pbf_octree_path_leaves(pbf_ctx *c, int nx, int ny, int nz, double Lx, double Ly, double Lz,
                                  int max_level, double radius, int n_tracks, const pbf_track *tracks,
                                  double s_lo, double s_hi, int32_t *leaves, int64_t capacity, int64_t *n_leaves)
{
    if (!n_leaves) return fail(c, PBF_EINVAL, "n_leaves is NULL");
    if (n_tracks < 0 || (n_tracks > 0 && !tracks)) return fail(c, PBF_EINVAL, "bad track list");
    const int n0[3] = {nx, ny, nz};
    const double L[3] = {Lx, Ly, Lz};
    std::vector<double> tr(8 * (size_t)n_tracks);
    for (int k = 0; k < n_tracks; ++k) {
        for (int d = 0; d < 3; ++d) {
            tr[8 * k + d] = tracks[k].x0[d];
            tr[8 * k + 3 + d] = tracks[k].x1[d];
        }
        tr[8 * k + 6] = tracks[k].speed;
        tr[8 * k + 7] = tracks[k].power;
    }
    std::vector<int32_t> out;
    std::string err;
    if (!oct_path_leaves(n0, L, max_level, radius, tr.data(), n_tracks, s_lo, s_hi, out, err))
        return fail(c, PBF_EINVAL, "%s", err.c_str());
    *n_leaves = (int64_t)(out.size() / 4);
    if (capacity < *n_leaves)
        return leaves ? fail(c, PBF_ENOMEM, "leaf array holds %lld leaves, %lld needed", (long long)capacity,
                             (long long)*n_leaves)
                      : PBF_OK;
    if (!leaves) return PBF_OK;
    std::copy(out.begin(), out.end(), leaves);
    return PBF_OK;
}

pbf_status pbf_octree_info(const pbf_ctx *c, int64_t *n_leaves, int64_t *n_hanging, int *max_level)
{
    if (!c) return fail(nullptr, PBF_EINVAL, "ctx is NULL");
    if (!c->has_mesh || !c->octree) return fail(const_cast<pbf_ctx *>(c), PBF_ESTATE, "no octree mesh");
    if (n_leaves) *n_leaves = c->oct.n_cells;
    if (n_hanging) *n_hanging = c->oct.n_hanging;
    if (max_level) *max_level = c->oct.maxl;
    return PBF_OK;
}

pbf_status pbf_dof_coords(const pbf_ctx *c, double *xyz)
{
    if (!c || !xyz) return fail(const_cast<pbf_ctx *>(c), PBF_EINVAL, "NULL argument");
    if (!c->has_mesh) return fail(const_cast<pbf_ctx *>(c), PBF_ESTATE, "no mesh");
    if (c->octree) {
        std::copy(c->oct.coords.begin(), c->oct.coords.end(), xyz);
        return PBF_OK;
    }
    const long long NX = nodes1(c, 0), NY = nodes1(c, 1), NZ = nodes1(c, 2);
    const double h[3] = {c->L[0] / c->nx / c->degree, c->L[1] / c->ny / c->degree, c->L[2] / c->nz / c->degree};
    for (long long k = 0; k < NZ; ++k)
        for (long long j = 0; j < NY; ++j)
            for (long long i = 0; i < NX; ++i) {
                double *x = xyz + 3 * (i + NX * (j + NY * k));
                x[0] = i * h[0];
                x[1] = j * h[1];
                x[2] = k * h[2];
            }
    return PBF_OK;
}

pbf_status pbf_mesh_info(const pbf_ctx *c, int64_t *nd, int64_t *nc, int64_t *nq, int64_t *nhl,
                         int64_t *nhc, int64_t *nhq)
{
    if (!c) return fail(nullptr, PBF_EINVAL, "pbf_mesh_info: ctx is NULL");
    if (!c->has_mesh) return fail(const_cast<pbf_ctx *>(c), PBF_ESTATE, "no mesh");
    const long long q = nq1(c);
    if (nd) *nd = alloc_dofs(c);
    if (nc) *nc = alloc_cells(c);
    if (nq) *nq = alloc_cells(c) * q * q * q;
    if (nhl) *nhl = c->hist_layers;
    if (nhc) *nhc = n_hist_cells(c);
    if (nhq) *nhq = n_hist_qp(c);
    return PBF_OK;
}

pbf_status pbf_set_active_layers(pbf_ctx *c, int nz_active)
{
    if (!c) return fail(nullptr, PBF_EINVAL, "ctx is NULL");
    if (!c->has_mesh || c->octree) return fail(c, PBF_ESTATE, "layer activation needs a box mesh");
    if (c->bound) return fail(c, PBF_ESTATE, "set the active layers before pbf_bind_device");
    const int nzf = c->growing ? c->nz_full : c->nz;
    if (nz_active < 1 || nz_active > nzf) return fail(c, PBF_EINVAL, "nz_active must be in [1, %d]", nzf);
    if (!c->growing) {
        c->nz_full = c->nz;
        c->Lz_full = c->L[2];
        c->growing = true;
    }
    c->nz = nz_active;
    c->L[2] = c->Lz_full * nz_active / c->nz_full;
    compute_history_layers(c);
    return PBF_OK;
}

pbf_status pbf_active_info(const pbf_ctx *c, int *nz_active, int64_t *n_active_dofs, double *Lz_active)
{
    if (!c) return fail(nullptr, PBF_EINVAL, "ctx is NULL");
    if (!c->has_mesh) return fail(const_cast<pbf_ctx *>(c), PBF_ESTATE, "no mesh");
    if (nz_active) *nz_active = c->nz;
    if (n_active_dofs) *n_active_dofs = n_dofs(c);
    if (Lz_active) *Lz_active = c->L[2];
    return PBF_OK;
}

pbf_status pbf_activate_layers(pbf_ctx *c, int nz_new, double T0, double *T, double *rc, void *stream)
{
    if (!c) return fail(nullptr, PBF_EINVAL, "ctx is NULL");
    pbf_status st = check_bound(c);
    if (st) return st;
    if (!c->growing) return fail(c, PBF_ESTATE, "not a growing box (pbf_set_active_layers before binding)");
    if (nz_new <= c->nz || nz_new > c->nz_full)
        return fail(c, PBF_EINVAL, "nz_new must be in [%d, %d]", c->nz + 1, c->nz_full);
    if (!T || (n_hist_qp(c) > 0 && !rc)) return fail(c, PBF_EINVAL, "NULL device array");
    if (!std::isfinite(T0)) return fail(c, PBF_EINVAL, "T0 must be finite");
    hipStream_t s = (hipStream_t)stream;
    const long long NXY = nodes1(c, 0) * nodes1(c, 1);
    const long long k_old = (long long)c->degree * c->nz, k_new = (long long)c->degree * nz_new;
    // new node planes k_old+1 .. k_new start at T0 (Section 2: activated parts start at T_0)
    PBF_HIP(c, launch_fill(T + NXY * (k_old + 1), T0, NXY * (k_new - k_old), s));
    const long long cpl = (long long)c->nx * c->ny;
    const int nz_old = c->nz;
    c->nz = nz_new;
    c->L[2] = c->Lz_full * nz_new / c->nz_full;
    compute_history_layers(c);
    // new cells: powder at the Gauss points within powder_depth of the new top
    if (n_hist_qp(c) > 0)
        PBF_HIP(c, launch_layer_history(c->degree, rc, n_hist_cells(c), cpl * nz_old, cpl * nz_new, (int)cpl,
                                        c->L[2] / c->nz, c->L[2], c->powder_depth, s));
    return PBF_OK;
}

pbf_status pbf_set_dirichlet(pbf_ctx *c, unsigned face_mask, double T_D)
{
    if (!c) return fail(nullptr, PBF_EINVAL, "pbf_set_dirichlet: ctx is NULL");
    if (face_mask > 63u) return fail(c, PBF_EINVAL, "face mask must use bits 0..5");
    if (!std::isfinite(T_D)) return fail(c, PBF_EINVAL, "T_D must be finite");
    c->dmask = face_mask;
    c->T_D = T_D;
    if (c->octree) {
        compute_history_layers(c);
        c->oct_flags_dirty = true;
    }
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
    const long long old_hist_cells = n_hist_cells(c);
    compute_history_layers(c);
    if (c->bound && (c->hist_layers != old_layers || n_hist_cells(c) != old_hist_cells))
        c->bound = false;  // sizes changed
    if (c->octree) c->oct_flags_dirty = true;
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

pbf_status pbf_set_surface_loss(pbf_ctx *c, const pbf_surface_loss *r)
{
    if (!c) return fail(nullptr, PBF_EINVAL, "ctx is NULL");
    SurfaceLoss q{};
    if (r && (r->emissivity != 0.0 || r->evap_on)) {
        if (!(r->emissivity >= 0 && std::isfinite(r->emissivity)) || !(r->T_inf >= 0 && std::isfinite(r->T_inf)))
            return fail(c, PBF_EINVAL, "need finite emissivity >= 0 and T_inf >= 0");
        if (r->evap_on && !(r->T_v > 0 && r->C_M > 0 && r->dT_max > 0 && r->C_P >= 0 && r->C_T >= 0 &&
                            r->h_v >= 0 && std::isfinite(r->T_v + r->C_M + r->dT_max + r->C_P + r->C_T + r->h_v +
                                                         r->T_h0)))
            return fail(c, PBF_EINVAL, "evaporation: need T_v, C_M, dT_max > 0 and C_P, C_T, h_v >= 0, all finite");
        const double sigma_S = 5.670374419e-8;  // W m^-2 K^-4 (exact in the 2019 SI)
        const double Ti2 = r->T_inf * r->T_inf;
        q.on = 1;
        q.evap = r->evap_on ? 1 : 0;
        q.eps_sigma = r->emissivity * sigma_S;
        q.Tinf4 = Ti2 * Ti2;
        q.Tv = r->T_v;
        q.inv_Tv = r->evap_on ? 1.0 / r->T_v : 0.0;
        q.Tmax = r->T_v + r->dT_max;
        q.CP82 = 0.82 * r->C_P;
        q.CT = r->C_T;
        q.CM = r->C_M;
        q.hv = r->h_v;
        q.Th0 = r->T_h0;
    }
    c->re = q;
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

// doubles of the CG-apply coefficient cache (boxes; octrees apply on the fly)
size_t picard_coef_count(const pbf_ctx *c)
{
    if (c->octree) return 0;
    const size_t nq = (size_t)(c->degree + 1) * (c->degree + 1) * (c->degree + 1);
    return (size_t)kCoefPicard * nq * (size_t)alloc_cells(c);
}

pbf_status pbf_workspace_bytes(const pbf_ctx *c, size_t *bytes)
{
    if (!c || !bytes) return fail(const_cast<pbf_ctx *>(c), PBF_EINVAL, "NULL argument");
    if (!c->has_mesh) return fail(const_cast<pbf_ctx *>(c), PBF_ESTATE, "no mesh");
    const size_t N = (size_t)alloc_dofs(c);
    size_t b = 0;
    b += align256(sizeof(Law<double>)) * 3 + align256(sizeof(Law<float>));
    const long long faces = slot_entries(c);
    if (faces > 0x7FFFFFFFLL)  // face nodes are indexed with 32-bit thread indices
        return fail(const_cast<pbf_ctx *>(c), PBF_EINVAL, "box too large: %lld column-face nodes", faces);
    b += align256(8 * (size_t)faces * sizeof(double));  // parity slots (boxes)
    b += 11 * align256(N * sizeof(double));       // f, C, v; implicit: y, diag, r, z, p, Ap, x, d
    b += align256(kRedBlocks * 4 * sizeof(double)); // reduction partials
    b += align256(64 * sizeof(double));           // device scalars
    b += align256(adjoint_tiles(c) * sizeof(double));  // adjoint tile partials
    b += align256(3 * kMaxProbes * sizeof(int)) + align256(4 * kMaxProbes * sizeof(double));
    b += align256(picard_coef_count(c) * sizeof(double));  // CG-apply coefficient cache (boxes)
    b += oct_tables(const_cast<pbf_ctx *>(c), nullptr);  // octree tables and element buffer
    if (c->precond == 1) {  // multigrid: fine smoother vectors and the coarse levels' workspaces
        b += 4 * align256(N * sizeof(double));
        for (pbf_ctx *l : c->mg) {
            size_t lb = 0;
            pbf_status st = pbf_workspace_bytes(l, &lb);
            if (st) return fail(const_cast<pbf_ctx *>(c), st, "multigrid level: %s", l->err.c_str());
            b += align256(lb);
        }
    }
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
    const size_t N = (size_t)alloc_dofs(c);
    char *p = (char *)workspace;
    c->d_law64 = (Law<double> *)p;
    p += align256(sizeof(Law<double>));
    c->d_lin64 = (Law<double> *)p;
    p += align256(sizeof(Law<double>));
    c->d_zero64 = (Law<double> *)p;
    p += align256(sizeof(Law<double>));
    c->d_law32 = (Law<float> *)p;
    p += align256(sizeof(Law<float>));
    c->d_slots = (double *)p;
    p += align256(8 * (size_t)slot_entries(c) * sizeof(double));
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
    p += align256(64 * sizeof(double));
    c->d_tiles = (double *)p;
    p += align256(adjoint_tiles(c) * sizeof(double));
    c->d_probe_cell = (int *)p;
    p += align256(3 * kMaxProbes * sizeof(int));
    c->d_probe_xi = (double *)p;
    c->d_probe_target = c->d_probe_xi + 3 * kMaxProbes;
    p += align256(4 * kMaxProbes * sizeof(double));
    c->d_coef = (double *)p;
    p += align256(picard_coef_count(c) * sizeof(double));
    c->probes_dirty = !c->probe_target.empty();
    c->bound = false;
    if (c->octree) {
        compute_history_layers(c);  // Dirichlet flags and history leaves for the current setup
        p += oct_tables(c, p);
        if ((st = oct_upload(c, (hipStream_t)stream, true))) return st;
    }
    if (c->precond == 1) {
        for (int k = 0; k < 4; ++k) {
            c->d_mg[k] = (double *)p;
            p += align256(N * sizeof(double));
        }
        for (pbf_ctx *l : c->mg) {
            size_t lb = 0;
            if ((st = pbf_workspace_bytes(l, &lb))) return fail(c, st, "multigrid level: %s", l->err.c_str());
            if ((st = pbf_bind_device(l, p, lb, stream))) return fail(c, st, "multigrid level: %s", l->err.c_str());
            p += align256(lb);
        }
    }
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
    if (!c->has_mesh) return fail(c, PBF_ESTATE, "no mesh: call pbf_mesh_box first");
    if (!c->has_material) return fail(c, PBF_ESTATE, "no material: call pbf_set_material first");
    // box meshes need no workspace here (the fills take their sizes as arguments)
    if (c->octree && !c->bound) return fail(c, PBF_ESTATE, "no device workspace: call pbf_bind_device first");
    pbf_status st = PBF_OK;
    if (!T) return fail(c, PBF_EINVAL, "T is NULL");
    if (n_hist_qp(c) > 0 && !rc) return fail(c, PBF_EINVAL, "rc is NULL but the mesh has history");
    if (!std::isfinite(T0)) return fail(c, PBF_EINVAL, "T0 must be finite");
    hipStream_t s = (hipStream_t)stream;
    c->T_init = T0;
    if (c->Tref != T0) {
        c->Tref = T0;
        c->laws_dirty = true;
    }
    if (c->bound && (st = upload_laws(c, s))) return st;
    PBF_HIP(c, launch_fill(T, T0, alloc_dofs(c), s));
    PBF_HIP(c, launch_init_dirichlet(T, geometry(c), c->T_D, s));
    if (c->growing) {
        if (n_hist_qp(c) > 0)
            PBF_HIP(c, launch_layer_history(c->degree, rc, n_hist_cells(c), 0, alloc_cells(c), c->nx * c->ny,
                                            c->L[2] / c->nz, c->L[2], c->powder_depth, s));
    } else if (n_hist_qp(c) > 0) {
        if (c->octree)
            PBF_HIP(c, launch_oct_init_history(c->od, c->degree, c->powder_depth, rc, s));
        else
            PBF_HIP(c, launch_init_history(rc, (int)n_hist_cells(c), nq1(c), c->powder_levels.data(),
                                           c->hist_layers, c->nx, c->ny, s));
    }
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
    if (c->octree && precision != PBF_PREC_FP64) return fail(c, PBF_EINVAL, "octree meshes run in FP64 only");
    hipStream_t s = (hipStream_t)stream;
    if ((st = upload_laws(c, s))) return st;
    double *cur = T, *nxt = T_tmp;
    for (int n = 0; n < n_steps; ++n) {
        const double t = t0 + n * dt;
        st = operator_pass(c, 0, precision, LAW_FULL, cur, nxt, nullptr, nullptr, rc, t, dt, s);
        if (st) return st;
        std::swap(cur, nxt);
    }
    if (cur != T) PBF_HIP(c, hipMemcpyAsync(T, cur, n_dofs(c) * sizeof(double), hipMemcpyDeviceToDevice, s));
    return PBF_OK;
}

pbf_status pbf_explicit_steps_noalloc(pbf_ctx *c, double *T, double *T_tmp, double *rc, double t0, double dt,
                                      int n_steps, int precision, size_t *scratch_bytes, void *stream)
{
    if (!c) return fail(nullptr, PBF_EINVAL, "ctx is NULL");
    if (!c->has_mesh) return fail(c, PBF_ESTATE, "no mesh: call pbf_mesh_box first");
    if (!c->has_material) return fail(c, PBF_ESTATE, "no material: call pbf_set_material first");
    if (c->octree) return fail(c, PBF_EMESH, "explicit steps without a workspace run on box meshes only");
    const long long faces = slot_entries(c);
    const size_t need = align256(sizeof(Law<double>)) * 3 + align256(sizeof(Law<float>)) +
                        align256(8 * (size_t)faces * sizeof(double));
    if (scratch_bytes) *scratch_bytes = need;
    if (need > kStaticScratchBytes)
        return fail(c, PBF_ENOMEM, "mesh needs %zu bytes of scratch; the static scratch holds %zu bytes", need,
                    kStaticScratchBytes);
    if (!T || !T_tmp || T == T_tmp) return fail(c, PBF_EINVAL, "T and T_tmp must be distinct device arrays");
    if (n_hist_qp(c) > 0 && !rc) return fail(c, PBF_EINVAL, "rc is NULL but the mesh has history");
    if (n_steps < 0) return fail(c, PBF_EINVAL, "n_steps must be >= 0");
    if (!(dt > 0) || !std::isfinite(t0)) return fail(c, PBF_EINVAL, "need dt > 0 and finite t0");
    if (precision != PBF_PREC_FP64 && precision != PBF_PREC_FP32)
        return fail(c, PBF_EINVAL, "precision must be 64 or 32");
    char *base = nullptr;
    pbf_status st = static_scratch(c, &base);
    if (st) return st;
    hipStream_t s = (hipStream_t)stream;
    ScratchBinding bind(c, base);
    if ((st = upload_laws(c, s))) return st;
    double *cur = T, *nxt = T_tmp;
    for (int n = 0; n < n_steps; ++n) {
        const double t = t0 + n * dt;
        st = operator_pass(c, 0, precision, LAW_FULL, cur, nxt, nullptr, nullptr, rc, t, dt, s);
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
    if (c->octree && precision != PBF_PREC_FP64) return fail(c, PBF_EINVAL, "octree meshes run in FP64 only");
    hipStream_t s = (hipStream_t)stream;
    if ((st = upload_laws(c, s))) return st;
    return operator_pass(c, 1, precision, LAW_FULL, T, nullptr, f, C, rc, t, 0.0, s);
}

pbf_status pbf_laplace_apply(pbf_ctx *c, const double *x, double *y, void *stream)
{
    if (!c) return fail(nullptr, PBF_EINVAL, "ctx is NULL");
    pbf_status st = check_bound(c);
    if (st) return st;
    if (c->octree) return fail(c, PBF_EMESH, "the Laplace reference operator runs on box meshes");
    if (!x || !y) return fail(c, PBF_EINVAL, "NULL device array");
    if (x == y) return fail(c, PBF_EINVAL, "x and y must not overlap");
    hipStream_t s = (hipStream_t)stream;
    if ((st = upload_laws(c, s))) return st;
    CellParams<double> pd = cell_params<double>(c, c->d_law64, false);
    pd.Tin = x;
    pd.fout = y;
    const CellParams<float> pf{};
    const bool timed = c->timing && (c->timing_seen++ % c->timing_every) == 0 && c->tev_used + 4 <= c->tev.size();
    hipEvent_t *ev = timed ? &c->tev[c->tev_used] : nullptr;
    PBF_HIP(c, launch_cells(c->degree, PBF_PREC_FP64, 2, column_height(), pd, pf, s, ev ? ev[0] : nullptr,
                            ev ? ev[1] : nullptr));
    HaloParams h = geometry(c);
    h.Tin = x;
    h.fout = y;
    const bool faces = h.GX + h.GY + h.GZ > 0;
    PBF_HIP(c, launch_halo(2, h, s, ev ? ev[2] : nullptr, ev ? ev[3] : nullptr));
    if (timed) {
        if (!faces) {
            PBF_HIP(c, hipEventRecord(ev[2], s));
            PBF_HIP(c, hipEventRecord(ev[3], s));
        }
        c->tev_used += 4;
    }
    return PBF_OK;
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
        st = operator_pass(c, 1, PBF_PREC_FP64, LAW_CRITICAL, c->d_v, nullptr, c->d_f, c->d_C, nullptr, 0.0,
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

pbf_status pbf_stability_dt(pbf_ctx *c, const double *v0, int iters, double *dt_crit, double *lambda_max,
                            void *stream)
{
    if (!c) return fail(nullptr, PBF_EINVAL, "ctx is NULL");
    if (!dt_crit) return fail(c, PBF_EINVAL, "dt_crit is NULL");
    double lam = 0.0;
    pbf_status st = pbf_stability_lambda(c, v0, iters, &lam, stream);
    if (st) return st;
    if (!(lam > 0.0) || !std::isfinite(lam))
        return fail(c, PBF_ENONFINITE, "stability estimate is not a positive finite eigenvalue (%g)", lam);
    *dt_crit = 2.0 / lam;
    if (lambda_max) *lambda_max = lam;
    return PBF_OK;
}

pbf_status pbf_set_implicit_preconditioner(pbf_ctx *c, int kind, int smoothing_degree, int coarse_degree)
{
    if (!c) return fail(nullptr, PBF_EINVAL, "ctx is NULL");
    if (kind != 0 && kind != 1) return fail(c, PBF_EINVAL, "kind must be 0 (Jacobi) or 1 (multigrid)");
    if (kind == 1) {
        if (!c->has_mesh || !c->has_material) return fail(c, PBF_ESTATE, "set the mesh and the material first");
        if (c->octree || c->growing) return fail(c, PBF_EMESH, "the multigrid preconditioner needs a full box mesh");
        if (smoothing_degree < 1 || smoothing_degree > 8 || coarse_degree < 1 || coarse_degree > 64)
            return fail(c, PBF_EINVAL, "smoothing degree in [1, 8], coarse degree in [1, 64]");
    }
    c->precond = kind;
    c->mg_smooth = smoothing_degree;
    c->mg_coarse = coarse_degree;
    c->bound = false;  // the workspace size changes
    if (kind == 1) return mg_build_levels(c);
    for (pbf_ctx *l : c->mg) pbf_destroy(l);
    c->mg.clear();
    return PBF_OK;
}

pbf_status pbf_set_newton_forcing(pbf_ctx *c, int kind)
{
    if (!c) return fail(nullptr, PBF_EINVAL, "ctx is NULL");
    if (kind != 0 && kind != 1) return fail(c, PBF_EINVAL, "kind must be 0 (fixed) or 1 (Eisenstat-Walker)");
    c->newton_forcing = kind;
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
    const HaloParams hp = geometry(c, picard_column_height(), kPicardResident);
    double *y = c->d_cg[0], *diag = c->d_cg[1], *r = c->d_cg[2], *z = c->d_cg[3], *p = c->d_cg[4],
           *Ap = c->d_cg[5], *x = c->d_cg[6], *d = c->d_cg[7];
    double *Ti = T_out;
    PBF_HIP(c, hipMemcpyAsync(Ti, T_n, N * sizeof(double), hipMemcpyDeviceToDevice, s));
    PBF_HIP(c, launch_init_dirichlet(Ti, ge, c->T_D, s));
    const Beam bm = beam_at(c, t + dt);
    // surface losses lagged at T_n (Section 3.2): f_RE(T_n) once per step
    const bool re = c->re.on != 0;
    if (re && (st = operator_pass(c, 1, PBF_PREC_FP64, LAW_SURFACE, T_n, nullptr, c->d_f, c->d_C, nullptr, t,
                                  0.0, s)))
        return st;
    int total = 0, it = 0;
    bool cg_fail = false, converged = false;
    double last_rel = 0.0;
    double hs[8];
    const bool mg = c->precond == 1 && !c->octree;
    std::vector<MgLevel> lev;
    if (mg) lev = mg_levels(c, T_n, Ti, diag, c->d_coef);
    for (it = 0; it < picard_max_it;) {
        // residual R(T^i) = C(T_n)(T^i - T_n)/dt + K(T^i) T^i - f_RE(T_n) - f_vol, and diag(A(T^i))
        PBF_HIP(c, launch_sub(d, Ti, T_n, N, s));
        if ((st = picard_pass(c, 0, hp, T_n, Ti, d, Ti, y, rc, dt, &bm, s))) return st;
        if (re) PBF_HIP(c, launch_sub(y, y, c->d_f, N, s));
        if ((st = picard_pass(c, 1, hp, T_n, Ti, nullptr, nullptr, diag, rc, dt, nullptr, s))) return st;
        if (!c->octree) {  // per-point coefficients of this iteration's CG applies
            PicardParams pc = picard_params(c, ge, T_n, Ti, nullptr, nullptr, nullptr, rc, dt, nullptr);
            pc.coef = c->d_coef;
            pc.ncells = (long long)c->nx * c->ny * c->nz;
            PBF_HIP(c, launch_picard_coef(c->degree, false, pc, s));
        }
        PBF_HIP(c, launch_cg_start(y, diag, r, z, p, x, c->d_partials, c->d_scal, ge, N, s));
        if (mg) {  // z = M^-1 r by a V-cycle, p = z, rz = r.z
            if ((st = mg_setup(c, lev, dt, s))) return st;
            if (it == 0 && (st = mg_eigen(c, lev, dt, s))) return st;
            if ((st = mg_precond(c, lev, r, z, dt, s))) return st;
            PBF_HIP(c, hipMemcpyAsync(p, z, N * sizeof(double), hipMemcpyDeviceToDevice, s));
            PBF_HIP(c, launch_dot_to(r, z, c->d_partials, c->d_scal + CG_RZ0, N, s));
        }
        PBF_HIP(c, hipMemcpyAsync(hs, c->d_scal + CG_RZ0, 6 * sizeof(double), hipMemcpyDeviceToHost, s));
        PBF_HIP(c, hipStreamSynchronize(s));
        const double bn = std::sqrt(hs[CG_BN2 - CG_RZ0]);
        double rr = hs[CG_RR - CG_RZ0];
        int k = 0, rz_old = CG_RZ0;
        last_rel = bn > 0 ? std::sqrt(rr) / bn : 0.0;
        while (bn > 0 && std::sqrt(rr) > cg_rtol * bn && k < cg_max_it) {
            if (c->octree) {
                if ((st = picard_pass(c, 0, hp, T_n, Ti, p, p, Ap, rc, dt, nullptr, s))) return st;
            } else {
                PicardParams pa = picard_params(c, ge, T_n, Ti, p, p, Ap, rc, dt, nullptr);
                pa.coef = c->d_coef;
                pa.ncells = (long long)c->nx * c->ny * c->nz;
                PBF_HIP(c, launch_picard_capply(c->degree, false, pa, ge, s));
            }
            PBF_HIP(c, launch_cg_pap(p, Ap, c->d_partials, c->d_scal, N, s));
            PBF_HIP(c, launch_cg_update(x, r, z, p, Ap, diag, c->d_partials, c->d_scal, rz_old, N, s));
            // |r|^2 into pinned memory; the next direction is computed while the
            // host waits for that read only (the direction is unused when the loop ends)
            if (!c->ev_read) PBF_HIP(c, hipEventCreateWithFlags(&c->ev_read, hipEventDisableTiming));
            if (!c->h_read)
                PBF_HIP(c, hipHostMalloc((void **)&c->h_read, (2 * kGmMax + 8) * sizeof(double), hipHostMallocDefault));
            PBF_HIP(c, hipMemcpyAsync(c->h_read, c->d_scal + CG_RR, sizeof(double), hipMemcpyDeviceToHost, s));
            PBF_HIP(c, hipEventRecord(c->ev_read, s));
            const int rz_new = rz_old == CG_RZ0 ? CG_RZ1 : CG_RZ0;
            if (mg) {  // z = M^-1 r, rz = r.z
                if ((st = mg_precond(c, lev, r, z, dt, s))) return st;
                PBF_HIP(c, launch_dot_to(r, z, c->d_partials, c->d_scal + rz_new, N, s));
            }
            PBF_HIP(c, launch_cg_direction(p, z, c->d_scal, rz_old, rz_new, N, s));
            PBF_HIP(c, hipEventSynchronize(c->ev_read));
            rr = c->h_read[0];
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
    st = operator_pass(c, 1, PBF_PREC_FP64, LAW_FULL, Ti, nullptr, c->d_f, c->d_C, rc, t + dt, 0.0, s);
    if (st) return st;
    if (cg_iters_total) *cg_iters_total = total;
    if (picard_iters) *picard_iters = it;
    if (final_rel_res) *final_rel_res = last_rel;
    if (cg_fail) return fail(c, PBF_ENOCONV, "CG did not reach the relative tolerance %g", cg_rtol);
    if (!converged) return fail(c, PBF_ENOCONV, "Picard did not converge in %d iterations", picard_max_it);
    return PBF_OK;
}

// ---- Newton step with restarted GMRES ----------------------------------------

struct NewtonWork {
    double *V, *partials, *h1, *h2, *hn, *y, *coef;
};

size_t newton_work_layout(long long N, long long ncoef, int restart, char *base, NewtonWork *w)
{
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char *p = base ? base + off : nullptr;
        off += align256(bytes);
        return (double *)p;
    };
    NewtonWork t{};
    t.V = take((size_t)(restart + 1) * N * sizeof(double));
    t.partials = take((size_t)kRedBlocks * kGmMax * sizeof(double));
    t.h1 = take(kGmMax * sizeof(double));
    t.h2 = take(kGmMax * sizeof(double));
    t.hn = take(kGmMax * sizeof(double));
    t.y = take(kGmMax * sizeof(double));
    t.coef = take((size_t)ncoef * sizeof(double));
    if (w) *w = t;
    return off;
}

long long newton_coef_count(const pbf_ctx *c)
{
    const long long nq = (long long)(c->degree + 1) * (c->degree + 1) * (c->degree + 1);
    return c->octree ? 0 : (long long)kCoefNewton * nq * alloc_cells(c);
}

pbf_status pbf_newton_work_bytes(pbf_ctx *c, int restart, size_t *bytes)
{
    if (!c || !bytes) return fail(c, PBF_EINVAL, "NULL argument");
    if (!c->has_mesh) return fail(c, PBF_ESTATE, "no mesh");
    if (restart < 1 || restart > kGmMax - 1) return fail(c, PBF_EINVAL, "restart must be in [1, %d]", kGmMax - 1);
    *bytes = newton_work_layout(n_dofs(c), newton_coef_count(c), restart, nullptr, nullptr);
    return PBF_OK;
}

pbf_status pbf_implicit_step_newton(pbf_ctx *c, const double *T_n, double *T_out, double *rc, double t, double dt,
                                    double lin_rtol, int restart, int lin_max_it, double newton_tol,
                                    int newton_max_it, void *work, size_t work_bytes, int *lin_iters_total,
                                    int *newton_iters, double *final_rel_res, void *stream)
{
    if (!c) return fail(nullptr, PBF_EINVAL, "ctx is NULL");
    pbf_status st = check_bound(c);
    if (st) return st;
    if (c->octree) return fail(c, PBF_ESTATE, "the Newton step needs a box mesh (use pbf_implicit_step)");
    if (!T_n || !T_out || T_n == T_out) return fail(c, PBF_EINVAL, "T_n and T_out must be distinct device arrays");
    if (n_hist_qp(c) > 0 && !rc) return fail(c, PBF_EINVAL, "rc is NULL but the mesh has history");
    if (!(dt > 0) || !std::isfinite(t)) return fail(c, PBF_EINVAL, "need dt > 0 and finite t");
    if (!(lin_rtol > 0) || lin_max_it < 1 || !(newton_tol > 0) || newton_max_it < 1)
        return fail(c, PBF_EINVAL, "tolerances must be > 0 and iteration limits >= 1");
    if (restart < 1 || restart > kGmMax - 1) return fail(c, PBF_EINVAL, "restart must be in [1, %d]", kGmMax - 1);
    const long long N = n_dofs(c);
    NewtonWork nw{};
    const size_t need = newton_work_layout(N, newton_coef_count(c), restart, (char *)work, &nw);
    if (!work || work_bytes < need || ((uintptr_t)work & 255))
        return fail(c, PBF_EINVAL, "work must be a 256-byte aligned device buffer of pbf_newton_work_bytes");
    hipStream_t s = (hipStream_t)stream;
    if ((st = upload_laws(c, s))) return st;
    const HaloParams ge = geometry(c);
    const HaloParams hp = geometry(c, picard_column_height(), kPicardResident);
    double *y = c->d_cg[0], *diag = c->d_cg[1], *r = c->d_cg[2], *z = c->d_cg[3], *b = c->d_cg[4],
           *w = c->d_cg[5], *x = c->d_cg[6], *d = c->d_cg[7];
    double *Ti = T_out, *V = nw.V;
    PBF_HIP(c, hipMemcpyAsync(Ti, T_n, N * sizeof(double), hipMemcpyDeviceToDevice, s));
    PBF_HIP(c, launch_init_dirichlet(Ti, ge, c->T_D, s));
    const Beam bm = beam_at(c, t + dt);
    const bool re = c->re.on != 0;
    if (re && (st = operator_pass(c, 1, PBF_PREC_FP64, LAW_SURFACE, T_n, nullptr, c->d_f, c->d_C, nullptr, t,
                                  0.0, s)))
        return st;
    const int m = restart;
    std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1), hc(m + 1), yy(m), h1(kGmMax), h2(kGmMax);
    auto norm2 = [&](const double *v, double *out) -> pbf_status {  // ||v||, synchronizing
        PBF_HIP(c, launch_mdot(v, v, 0, 1, nw.partials, nw.hn, N, s));
        double v2 = 0.0;
        PBF_HIP(c, hipMemcpyAsync(&v2, nw.hn, sizeof(double), hipMemcpyDeviceToHost, s));
        PBF_HIP(c, hipStreamSynchronize(s));
        *out = std::sqrt(v2);
        return PBF_OK;
    };
    int total = 0, it = 0;
    bool lin_fail = false, converged = false;
    double last_rel = 0.0;
    const bool mg = c->precond == 1;
    std::vector<MgLevel> lev;
    if (mg) lev = mg_levels(c, T_n, Ti, diag, nw.coef);  // the symmetric part of the cached Jacobian
    double bn_prev = 0.0, eta_prev = 0.1;
    for (it = 0; it < newton_max_it;) {
        // residual R(T^i) = C(T_n)(T^i - T_n)/dt + K(T^i) T^i - f_RE(T_n) - f_vol; b = -R
        PBF_HIP(c, launch_sub(d, Ti, T_n, N, s));
        if ((st = picard_pass(c, 0, hp, T_n, Ti, d, Ti, y, rc, dt, &bm, s))) return st;
        if (re) PBF_HIP(c, launch_sub(y, y, c->d_f, N, s));
        PBF_HIP(c, launch_neg(b, y, N, s));
        if ((st = picard_pass(c, 1, hp, T_n, Ti, nullptr, nullptr, diag, rc, dt, nullptr, s))) return st;
        PicardParams pj = picard_params(c, ge, T_n, Ti, nullptr, nullptr, nullptr, rc, dt, nullptr);
        pj.coef = nw.coef;
        pj.ncells = (long long)c->nx * c->ny * c->nz;
        PBF_HIP(c, launch_picard_coef(c->degree, true, pj, s));
        auto japply = [&](const double *xin, double *yout) -> pbf_status {  // y = J(T^i) x, cached
            PicardParams pa = pj;
            pa.x1 = pa.x2 = xin;
            pa.yout = yout;
            PBF_HIP(c, launch_picard_capply(c->degree, true, pa, ge, s));
            return PBF_OK;
        };
        if (mg) {
            if ((st = mg_setup(c, lev, dt, s))) return st;
            if (it == 0 && (st = mg_eigen(c, lev, dt, s))) return st;
        }
        // GMRES(m) from x = 0 on J(T^i) x = b, Jacobi (or the multigrid V-cycle of
        // the symmetric part) on the right
        PBF_HIP(c, launch_fill(x, 0.0, N, s));
        PBF_HIP(c, hipMemcpyAsync(r, b, N * sizeof(double), hipMemcpyDeviceToDevice, s));
        double bn = 0.0, rn = 0.0;
        if ((st = norm2(b, &bn))) return st;
        rn = bn;
        // forcing term of this Newton system: lin_rtol, or (Eisenstat-Walker, choice 2)
        // eta = 0.9 (|R_k| / |R_k-1|)^2 safeguarded by 0.9 eta_k-1^2 when that exceeds
        // 0.1, capped at 0.1 and floored at lin_rtol
        double eta = lin_rtol;
        if (c->newton_forcing == 1) {
            if (it == 0) eta = 0.1;
            else {
                const double ratio = bn_prev > 0 ? bn / bn_prev : 1.0;
                eta = 0.9 * ratio * ratio;
                const double guard = 0.9 * eta_prev * eta_prev;
                if (guard > 0.1) eta = std::max(eta, guard);
                eta = std::min(eta, 0.1);
            }
            eta = std::max(eta, lin_rtol);
        }
        bn_prev = bn;
        eta_prev = eta;
        int k = 0;
        while (bn > 0 && rn > eta * bn && k < lin_max_it) {
            PBF_HIP(c, launch_div_scalar(V, r, rn, N, s));
            std::fill(g.begin(), g.end(), 0.0);
            g[0] = rn;
            int j;
            for (j = 0; j < m && k < lin_max_it; ++j) {
                double *Vj = V + (size_t)j * N, *Vn = V + (size_t)(j + 1) * N;
                if (mg) {
                    if ((st = mg_precond(c, lev, Vj, z, dt, s))) return st;
                } else {
                    PBF_HIP(c, launch_div(z, Vj, diag, N, s));
                }
                if ((st = japply(z, w))) return st;
                // classical Gram-Schmidt, twice
                PBF_HIP(c, launch_mdot(w, V, N, j + 1, nw.partials, nw.h1, N, s));
                PBF_HIP(c, launch_maxpy(w, V, N, j + 1, nw.h1, N, s));
                PBF_HIP(c, launch_mdot(w, V, N, j + 1, nw.partials, nw.h2, N, s));
                PBF_HIP(c, launch_maxpy(w, V, N, j + 1, nw.h2, N, s));
                PBF_HIP(c, launch_mdot(w, w, 0, 1, nw.partials, nw.hn, N, s));
                // both projections and |w|^2 into pinned memory, one wait
                if (!c->h_read)
                    PBF_HIP(c, hipHostMalloc((void **)&c->h_read, (2 * kGmMax + 8) * sizeof(double),
                                             hipHostMallocDefault));
                double *pin = c->h_read;
                PBF_HIP(c, hipMemcpyAsync(pin, nw.h1, (j + 1) * sizeof(double), hipMemcpyDeviceToHost, s));
                PBF_HIP(c, hipMemcpyAsync(pin + kGmMax, nw.h2, (j + 1) * sizeof(double), hipMemcpyDeviceToHost, s));
                PBF_HIP(c, hipMemcpyAsync(pin + 2 * kGmMax, nw.hn, sizeof(double), hipMemcpyDeviceToHost, s));
                PBF_HIP(c, hipStreamSynchronize(s));
                std::copy(pin, pin + j + 1, h1.begin());
                std::copy(pin + kGmMax, pin + kGmMax + j + 1, h2.begin());
                const double hn = std::sqrt(pin[2 * kGmMax]);
                ++k;
                for (int q = 0; q <= j; ++q) hc[q] = h1[q] + h2[q];
                if (hn > 0) PBF_HIP(c, launch_div_scalar(Vn, w, hn, N, s));
                else PBF_HIP(c, launch_fill(Vn, 0.0, N, s));
                for (int q = 0; q < j; ++q) {  // previous rotations
                    const double a = cs[q] * hc[q] + sn[q] * hc[q + 1];
                    hc[q + 1] = -sn[q] * hc[q] + cs[q] * hc[q + 1];
                    hc[q] = a;
                }
                const double den = std::sqrt(hc[j] * hc[j] + hn * hn);
                cs[j] = den > 0 ? hc[j] / den : 1.0;
                sn[j] = den > 0 ? hn / den : 0.0;
                hc[j] = den;
                g[j + 1] = -sn[j] * g[j];
                g[j] = cs[j] * g[j];
                for (int q = 0; q <= j; ++q) H[(size_t)q * m + j] = hc[q];
                if (std::fabs(g[j + 1]) <= eta * bn || hn == 0.0) {
                    ++j;
                    break;
                }
            }
            for (int q = j - 1; q >= 0; --q) {  // back substitution
                double sum = g[q];
                for (int l = q + 1; l < j; ++l) sum -= H[(size_t)q * m + l] * yy[l];
                yy[q] = sum / H[(size_t)q * m + q];
            }
            if (mg) {  // x += M^-1 (V y): t = 0 - V (-y), z = M^-1 t
                std::vector<double> ny(j);
                for (int q = 0; q < j; ++q) ny[q] = -yy[q];
                PBF_HIP(c, hipMemcpyAsync(nw.y, ny.data(), j * sizeof(double), hipMemcpyHostToDevice, s));
                PBF_HIP(c, launch_fill(c->d_v, 0.0, N, s));
                PBF_HIP(c, launch_maxpy(c->d_v, V, N, j, nw.y, N, s));
                if ((st = mg_precond(c, lev, c->d_v, z, dt, s))) return st;
                PBF_HIP(c, launch_axpy(x, 1.0, z, N, s));
                PBF_HIP(c, hipStreamSynchronize(s));  // ny is read by the copy
            } else {
                PBF_HIP(c, hipMemcpyAsync(nw.y, yy.data(), j * sizeof(double), hipMemcpyHostToDevice, s));
                PBF_HIP(c, launch_gm_update(x, V, N, j, nw.y, diag, N, s));
            }
            if ((st = japply(x, w))) return st;
            PBF_HIP(c, launch_sub(r, b, w, N, s));
            if ((st = norm2(r, &rn))) return st;
        }
        total += k;
        last_rel = bn > 0 ? rn / bn : 0.0;
        if (bn > 0 && rn > eta * bn) lin_fail = true;
        PBF_HIP(c, launch_picard_update(Ti, x, c->d_partials, c->d_scal, ge, N, s));
        double dmax = 0.0;
        PBF_HIP(c, hipMemcpyAsync(&dmax, c->d_scal + CG_DMAX, sizeof(double), hipMemcpyDeviceToHost, s));
        PBF_HIP(c, hipStreamSynchronize(s));
        ++it;
        if (!std::isfinite(dmax)) return fail(c, PBF_ENONFINITE, "non-finite Newton update");
        if (dmax <= newton_tol) {
            converged = true;
            break;
        }
    }
    st = operator_pass(c, 1, PBF_PREC_FP64, LAW_FULL, Ti, nullptr, c->d_f, c->d_C, rc, t + dt, 0.0, s);
    if (st) return st;
    if (lin_iters_total) *lin_iters_total = total;
    if (newton_iters) *newton_iters = it;
    if (final_rel_res) *final_rel_res = last_rel;
    if (lin_fail) return fail(c, PBF_ENOCONV, "GMRES did not reach the relative tolerance %g", lin_rtol);
    if (!converged) return fail(c, PBF_ENOCONV, "Newton did not converge in %d iterations", newton_max_it);
    return PBF_OK;
}

pbf_status pbf_set_probes(pbf_ctx *c, int n, const double *pts, const double *targets, void *stream)
{
    if (!c) return fail(nullptr, PBF_EINVAL, "ctx is NULL");
    if (c->octree) return fail(const_cast<pbf_ctx *>(c), PBF_ESTATE, "probes and the adjoint need a box mesh");
    if (!c->has_mesh) return fail(c, PBF_ESTATE, "no mesh");
    if (n < 0 || n > kMaxProbes) return fail(c, PBF_EINVAL, "number of probes must be in [0, %d]", kMaxProbes);
    if (n > 0 && !pts) return fail(c, PBF_EINVAL, "pts is NULL");
    std::vector<int> cell(3 * (size_t)n);
    std::vector<double> xi(3 * (size_t)n), tgt((size_t)n, 0.0);
    const int nc[3] = {c->nx, c->ny, c->nz};
    for (int p = 0; p < n; ++p) {
        for (int d = 0; d < 3; ++d) {
            const double tol = 1e-12 * c->L[d];  // points on a face up to rounding
            if (!(pts[3 * p + d] >= -tol && pts[3 * p + d] <= c->L[d] + tol))
                return fail(c, PBF_EINVAL, "probe %d lies outside the box", p);
            const double x = std::min(std::max(pts[3 * p + d], 0.0), c->L[d]);
            const double h = c->L[d] / nc[d];
            const double sx = x / h;
            int ci = (int)std::floor(sx);
            if (ci > 0 && (double)ci == sx) ci -= 1;  // shared face: lower cell
            ci = std::min(std::max(ci, 0), nc[d] - 1);
            cell[3 * p + d] = ci;
            xi[3 * p + d] = sx - ci;
        }
        if (targets) {
            if (!std::isfinite(targets[p])) return fail(c, PBF_EINVAL, "target %d is not finite", p);
            tgt[p] = targets[p];
        }
    }
    c->probe_cell = cell;
    c->probe_xi = xi;
    c->probe_target = tgt;
    c->probes_dirty = true;
    if (c->bound) return upload_probes(c, (hipStream_t)stream);
    return PBF_OK;
}

pbf_status pbf_probe(pbf_ctx *c, const double *T, double *vals, void *stream)
{
    if (!c) return fail(nullptr, PBF_EINVAL, "ctx is NULL");
    pbf_status st = check_bound(c);
    if (st) return st;
    if (!T || (!vals && !c->probe_target.empty())) return fail(c, PBF_EINVAL, "NULL device array");
    hipStream_t s = (hipStream_t)stream;
    if ((st = upload_probes(c, s))) return st;
    PBF_HIP(c, launch_probe_values(probe_set(c), T, vals, s));
    return PBF_OK;
}

pbf_status pbf_objective(pbf_ctx *c, const double *T, double *J, double *lam, void *stream)
{
    if (!c) return fail(nullptr, PBF_EINVAL, "ctx is NULL");
    pbf_status st = check_bound(c);
    if (st) return st;
    if (!T || !J || !lam) return fail(c, PBF_EINVAL, "NULL device array");
    hipStream_t s = (hipStream_t)stream;
    if ((st = upload_probes(c, s))) return st;
    PBF_HIP(c, launch_objective(probe_set(c), T, J, lam, n_dofs(c), s));
    return PBF_OK;
}

pbf_status pbf_adjoint_step(pbf_ctx *c, const double *T_n, const double *T_next, const double *rc_prev,
                            const double *lam_next, double *lam, double *mu, double t_n, double dt, double *dJdW,
                            void *stream)
{
    if (!c) return fail(nullptr, PBF_EINVAL, "ctx is NULL");
    if (c->re.on) return fail(c, PBF_ESTATE, "the adjoint does not cover surface losses (pbf_set_surface_loss)");
    if (c->growing) return fail(c, PBF_ESTATE, "the adjoint needs a fixed mesh (no layer activation)");
    if (c->octree) return fail(const_cast<pbf_ctx *>(c), PBF_ESTATE, "probes and the adjoint need a box mesh");
    pbf_status st = check_bound(c);
    if (st) return st;
    if (!T_n || !T_next || !lam_next || !lam) return fail(c, PBF_EINVAL, "NULL device array");
    if (lam == lam_next) return fail(c, PBF_EINVAL, "lam and lam_next must be distinct arrays");
    if (n_hist_qp(c) > 0 && (!rc_prev || !mu))
        return fail(c, PBF_EINVAL, "rc_prev and mu are required when the mesh has history");
    if (!c->tracks.empty() && !dJdW) return fail(c, PBF_EINVAL, "dJdW is NULL");
    if (!(dt > 0) || !std::isfinite(t_n)) return fail(c, PBF_EINVAL, "need dt > 0 and finite t_n");
    hipStream_t s = (hipStream_t)stream;
    if ((st = upload_laws(c, s))) return st;
    return adjoint_step(c, T_n, T_next, n_hist_qp(c) > 0 ? rc_prev : nullptr, lam_next, lam,
                        n_hist_qp(c) > 0 ? mu : nullptr, t_n, dt, dJdW, s);
}

pbf_status pbf_revolve_schedule(int n_steps, int n_snaps, pbf_revolve_action *actions, int max_actions,
                                int *n_actions, int64_t *n_advances)
{
    if (n_steps < 1 || n_steps > (1 << 24) || n_snaps < 1)
        return fail(nullptr, PBF_EINVAL, "need 1 <= n_steps <= 2^24 and n_snaps >= 1");
    std::vector<pbf_revolve_action> acts;
    long long adv = 0;
    if (!revolve_schedule(n_steps, n_snaps, acts, &adv)) return fail(nullptr, PBF_EINVAL, "bad schedule request");
    if (n_actions) *n_actions = (int)acts.size();
    if (n_advances) *n_advances = adv;
    if (actions) {
        if ((size_t)max_actions < acts.size())
            return fail(nullptr, PBF_EINVAL, "max_actions %d < %zu actions", max_actions, acts.size());
        std::copy(acts.begin(), acts.end(), actions);
    }
    return PBF_OK;
}

pbf_status pbf_adjoint_work_bytes(const pbf_ctx *c, int n_snaps, size_t *bytes)
{
    if (!c || !bytes) return fail(const_cast<pbf_ctx *>(c), PBF_EINVAL, "NULL argument");
    if (c->octree) return fail(const_cast<pbf_ctx *>(c), PBF_ESTATE, "probes and the adjoint need a box mesh");
    if (!c->has_mesh) return fail(const_cast<pbf_ctx *>(c), PBF_ESTATE, "no mesh");
    if (n_snaps < 1) return fail(const_cast<pbf_ctx *>(c), PBF_EINVAL, "n_snaps must be >= 1");
    *bytes = grad_layout(c, n_snaps, nullptr).bytes;
    return PBF_OK;
}

// The problem parameters that the forward sweep, the replays and the reverse
// steps of a gradient evaluation read, flattened in a fixed order: a backward
// sweep may only run on the problem its forward sweep saw.
static std::vector<double> grad_problem(const pbf_ctx *c)
{
    std::vector<double> v;
    v.push_back(c->n_bp);
    for (int i = 0; i < c->n_bp; ++i) {
        v.push_back(c->T_bp[i]);
        v.push_back(c->k_bp[i]);
        v.push_back(c->cp_bp[i]);
    }
    for (double x : {c->rho, c->T_s, c->T_l, c->latent, c->phi, c->powder_depth, double(c->laser_kind), c->radius,
                     c->absorptivity, c->h_powder, c->t_start, double(c->dmask), c->T_D})
        v.push_back(x);
    for (const pbf_track &t : c->tracks) {
        for (int d = 0; d < 3; ++d) {
            v.push_back(t.x0[d]);
            v.push_back(t.x1[d]);
        }
        v.push_back(t.speed);
        v.push_back(t.power);
    }
    for (int x : c->probe_cell) v.push_back(x);
    v.insert(v.end(), c->probe_xi.begin(), c->probe_xi.end());
    v.insert(v.end(), c->probe_target.begin(), c->probe_target.end());
    return v;
}

static bool same_bits(const std::vector<double> &a, const std::vector<double> &b)
{
    return a.size() == b.size() && (a.empty() || std::memcmp(a.data(), b.data(), a.size() * sizeof(double)) == 0);
}

static pbf_status check_grad_args(pbf_ctx *c, double dt, int n_steps, int n_snaps, void *work, size_t work_bytes)
{
    pbf_status st = check_bound(c);
    if (st) return st;
    if (c->octree) return fail(c, PBF_ESTATE, "probes and the adjoint need a box mesh");
    if (!(dt > 0)) return fail(c, PBF_EINVAL, "dt must be > 0");
    if (n_steps < 1 || n_steps > (1 << 24)) return fail(c, PBF_EINVAL, "n_steps must be in [1, 2^24]");
    if (n_snaps < 1) return fail(c, PBF_EINVAL, "n_snaps must be >= 1");
    if (!work || ((uintptr_t)work & 255) != 0) return fail(c, PBF_EINVAL, "work must be 256-byte aligned device memory");
    const size_t need = grad_layout(c, n_snaps, nullptr).bytes;
    if (work_bytes < need) return fail(c, PBF_ENOMEM, "work buffer too small: %zu < %zu bytes", work_bytes, need);
    return PBF_OK;
}

pbf_status pbf_gradient_forward(pbf_ctx *c, const double *T0, const double *rc0, double t0, double dt,
                                int n_steps, int n_snaps, void *work, size_t work_bytes, double *T_N,
                                double *J, void *stream)
{
    if (!c) return fail(nullptr, PBF_EINVAL, "ctx is NULL");
    if (c->re.on) return fail(c, PBF_ESTATE, "the adjoint does not cover surface losses (pbf_set_surface_loss)");
    if (c->growing) return fail(c, PBF_ESTATE, "the adjoint needs a fixed mesh (no layer activation)");
    pbf_status st = check_grad_args(c, dt, n_steps, n_snaps, work, work_bytes);
    if (st) return st;
    if (!T0 || (n_hist_qp(c) > 0 && !rc0)) return fail(c, PBF_EINVAL, "NULL initial state");
    if (!std::isfinite(t0)) return fail(c, PBF_EINVAL, "t0 must be finite");
    hipStream_t s = (hipStream_t)stream;
    if ((st = upload_laws(c, s))) return st;
    if ((st = upload_probes(c, s))) return st;
    c->grad.valid = false;
    std::vector<pbf_revolve_action> acts;
    long long adv = 0;
    revolve_schedule(n_steps, n_snaps, acts, &adv);
    size_t first_turn = 0;
    while (first_turn < acts.size() && acts[first_turn].kind != PBF_ACT_TURN) ++first_turn;
    const GradWork w = grad_layout(c, n_snaps, (char *)work);
    const size_t N = (size_t)n_dofs(c), H = (size_t)n_hist_qp(c);
    PBF_HIP(c, hipMemcpyAsync(w.B[0], T0, N * sizeof(double), hipMemcpyDeviceToDevice, s));
    if (H) PBF_HIP(c, hipMemcpyAsync(w.rcur, rc0, H * sizeof(double), hipMemcpyDeviceToDevice, s));
    std::vector<double> P(std::max<size_t>(c->tracks.size(), 1), 0.0);
    for (size_t k = 0; k < c->tracks.size(); ++k) P[k] = c->tracks[k].power;
    PBF_HIP(c, hipMemcpyAsync(w.powers, P.data(), P.size() * sizeof(double), hipMemcpyHostToDevice, s));
    PBF_HIP(c, hipStreamSynchronize(s));
    GradState g;
    g.cur = w.B[0];
    double *lam = w.lam, *lam2 = w.lam2;
    if ((st = run_actions(c, acts, 0, first_turn, w, g, lam, lam2, t0, dt, s))) return st;
    // last step (l-1 -> l) on a copy of the history; T_N is T_{n+1} of the first reverse step
    if (H) PBF_HIP(c, hipMemcpyAsync(w.rtmp, w.rcur, H * sizeof(double), hipMemcpyDeviceToDevice, s));
    double *TN = free_buffer(w, g);
    st = operator_pass(c, 0, PBF_PREC_FP64, LAW_FULL, g.cur, TN, nullptr, nullptr, H ? w.rtmp : nullptr,
                       t0 + (n_steps - 1) * dt, dt, s);
    if (st) return st;
    g.next = TN;
    PBF_HIP(c, launch_objective(probe_set(c), TN, w.J, w.lam, (long long)N, s));
    if (T_N) PBF_HIP(c, hipMemcpyAsync(T_N, TN, N * sizeof(double), hipMemcpyDeviceToDevice, s));
    if (J) PBF_HIP(c, hipMemcpyAsync(J, w.J, sizeof(double), hipMemcpyDeviceToDevice, s));
    c->grad.work = work;
    c->grad.n_steps = n_steps;
    c->grad.n_snaps = n_snaps;
    c->grad.t0 = t0;
    c->grad.dt = dt;
    c->grad.cur = g.cur;
    c->grad.next = g.next;
    c->grad.problem = grad_problem(c);
    c->grad.valid = true;
    return PBF_OK;
}

pbf_status pbf_gradient_backward(pbf_ctx *c, double t0, double dt, int n_steps, int n_snaps, void *work,
                                 size_t work_bytes, double *dJdW, double *dJdP, double *dJdA, double *lam0,
                                 int64_t *n_advances, void *stream)
{
    if (!c) return fail(nullptr, PBF_EINVAL, "ctx is NULL");
    if (c->re.on) return fail(c, PBF_ESTATE, "the adjoint does not cover surface losses (pbf_set_surface_loss)");
    if (c->growing) return fail(c, PBF_ESTATE, "the adjoint needs a fixed mesh (no layer activation)");
    pbf_status st = check_grad_args(c, dt, n_steps, n_snaps, work, work_bytes);
    if (st) return st;
    if (!c->grad.valid || c->grad.work != work || c->grad.n_steps != n_steps || c->grad.n_snaps != n_snaps ||
        c->grad.t0 != t0 || c->grad.dt != dt)
        return fail(c, PBF_ESTATE, "no matching forward sweep: call pbf_gradient_forward with the same arguments");
    if (!same_bits(c->grad.problem, grad_problem(c)))
        return fail(c, PBF_ESTATE,
                    "the problem changed since pbf_gradient_forward (material, laser, track powers, absorptivity, "
                    "boundary or probes): restore it or run the forward sweep again");
    c->grad.valid = false;  // the reversal consumes the forward state
    hipStream_t s = (hipStream_t)stream;
    if ((st = upload_laws(c, s))) return st;
    std::vector<pbf_revolve_action> acts;
    long long adv = 0;
    revolve_schedule(n_steps, n_snaps, acts, &adv);
    size_t first_turn = 0;
    while (first_turn < acts.size() && acts[first_turn].kind != PBF_ACT_TURN) ++first_turn;
    const GradWork w = grad_layout(c, n_snaps, (char *)work);
    const size_t N = (size_t)n_dofs(c), H = (size_t)n_hist_qp(c), K = c->tracks.size();
    if (H) PBF_HIP(c, launch_fill(w.mu, 0.0, (long long)H, s));
    PBF_HIP(c, launch_fill(w.dJdW, 0.0, (long long)std::max<size_t>(K, 1), s));
    GradState g;
    g.cur = c->grad.cur;
    g.next = c->grad.next;
    g.step = n_steps - 1;
    double *lam = w.lam, *lam2 = w.lam2;
    if ((st = run_actions(c, acts, first_turn, acts.size(), w, g, lam, lam2, t0, dt, s))) return st;
    if (K > 0) {
        if (dJdP || dJdA) PBF_HIP(c, launch_adjoint_params(w.dJdW, w.powers, c->absorptivity, (int)K, dJdP, dJdA, s));
        if (dJdW) PBF_HIP(c, hipMemcpyAsync(dJdW, w.dJdW, K * sizeof(double), hipMemcpyDeviceToDevice, s));
    } else if (dJdA) {
        PBF_HIP(c, launch_fill(dJdA, 0.0, 1, s));
    }
    if (lam0) PBF_HIP(c, hipMemcpyAsync(lam0, lam, N * sizeof(double), hipMemcpyDeviceToDevice, s));
    if (n_advances) *n_advances = adv;
    return PBF_OK;
}

pbf_status pbf_energy(pbf_ctx *c, const double *T_prev, const double *T, const double *rc, double t,
                      double dt, double out[4], void *stream)
{
    if (!c) return fail(nullptr, PBF_EINVAL, "ctx is NULL");
    pbf_status st = check_bound(c);
    if (st) return st;
    if (!T_prev || !T || !out) return fail(c, PBF_EINVAL, "NULL argument");
    if (n_hist_qp(c) > 0 && !rc) return fail(c, PBF_EINVAL, "rc is NULL but the mesh has history");
    if (!(dt > 0) || !std::isfinite(t)) return fail(c, PBF_EINVAL, "need dt > 0 and finite t");
    hipStream_t s = (hipStream_t)stream;
    if ((st = upload_laws(c, s))) return st;
    const long long N = n_dofs(c);
    // f and C~ of the step from T_prev (history read only), then the source alone
    st = operator_pass(c, 1, PBF_PREC_FP64, LAW_FULL, T_prev, nullptr, c->d_f, c->d_C,
                       const_cast<double *>(rc), t, 0.0, s, false);
    if (st) return st;
    st = operator_pass(c, 1, PBF_PREC_FP64, LAW_SOURCE, T_prev, nullptr, c->d_v, c->d_cg[0], nullptr, t,
                       0.0, s);
    if (st) return st;
    PBF_HIP(c, launch_energy(T_prev, T, c->d_f, c->d_v, c->d_C, c->d_partials, c->d_scal, geometry(c), N, s));
    double e[3];
    PBF_HIP(c, hipMemcpyAsync(e, c->d_scal + SC_ENERGY, sizeof e, hipMemcpyDeviceToHost, s));
    PBF_HIP(c, hipStreamSynchronize(s));
    out[0] = e[0];
    out[1] = e[1];
    out[2] = e[2];
    out[3] = e[0] - dt * (e[1] - e[2]);
    return PBF_OK;
}

pbf_status pbf_check_finite(pbf_ctx *c, const double *x, int64_t n, int *ok, double *maxabs, void *stream)
{
    if (!c) return fail(nullptr, PBF_EINVAL, "ctx is NULL");
    pbf_status st = check_bound(c);
    if (st) return st;
    if (!x || n < 1) return fail(c, PBF_EINVAL, "need a device array of n >= 1 values");
    hipStream_t s = (hipStream_t)stream;
    PBF_HIP(c, launch_finite(x, c->d_partials, c->d_scal, (long long)n, s));
    double r[2];
    PBF_HIP(c, hipMemcpyAsync(r, c->d_scal + SC_FINITE, sizeof r, hipMemcpyDeviceToHost, s));
    PBF_HIP(c, hipStreamSynchronize(s));
    if (ok) *ok = r[0] == 0.0;
    if (maxabs) *maxabs = r[1];
    return r[0] == 0.0 ? PBF_OK : fail(c, PBF_ENONFINITE, "%.0f non-finite values", r[0]);
}

static pbf_status prepare_remesh(pbf_ctx *c, int64_t n_leaves, const int32_t *leaves, int64_t new_top, size_t *bytes,
                                 int64_t *new_n_dofs, int64_t *new_n_hist_qp)
{
    c->pending.ready = false;
    const OctMesh &om = c->oct;
    OctMesh nm;
    std::string err;
    if (!oct_build(nm, c->degree, om.maxl, om.n0, om.L, n_leaves, leaves, err, new_top))
        return fail(c, PBF_EMESH, "%s", err.c_str());
    nm.growing = om.growing;
    oct_finish(nm, c->dmask, c->powder_depth);
    const int P = c->degree, N1 = P + 1;
    const bool grow = om.growing;
    // new dofs: containing old leaf and reference coordinates (growing builds:
    // dofs above the old top are activated, cell -1)
    c->pending.cell.resize(nm.n_dofs);
    c->pending.xi.assign(3 * nm.n_dofs, 0.0);
    for (int64_t i = 0; i < nm.n_dofs; ++i) {
        if (grow && nm.dof_key[3 * i + 2] > om.top * P) {
            c->pending.cell[i] = -1;
            continue;
        }
        double x[3];
        for (int d = 0; d < 3; ++d) x[d] = double(nm.dof_key[3 * i + d]) / P;
        const int32_t e = oct_locate(om, x, &c->pending.xi[3 * i]);
        if (e < 0) return fail(c, PBF_EMESH, "new dof outside the old mesh");
        c->pending.cell[i] = e;
    }
    // new history points.  Scan-following meshes: the nearest old Gauss point of
    // the containing old leaf if that point lies in the powder layer, else the
    // initial value.  Growing builds: points above the old top start as powder
    // (initial value), points of a coarsened parent take the minimum over the
    // points of its old children, the others the nearest old Gauss point of the
    // containing old leaf.
    auto gp = [&](int q) { return P == 1 ? Tables<1>::gp(q) : Tables<2>::gp(q); };
    const int64_t nq = (int64_t)N1 * N1 * N1;
    const double ztop_old = (double)om.top * om.unit[2], ztop_new = (double)nm.top * nm.unit[2];
    c->pending.src.assign(nq * nm.n_hist_cells, -2);
    c->pending.grp_start.assign(1, 0);
    c->pending.grp_idx.clear();
    for (int64_t e = 0; e < nm.n_cells; ++e) {
        const int32_t hc = nm.cell_hist[e];
        if (hc < 0) continue;
        const int ln = nm.leaf[4 * e];
        const double s = (double)(1LL << (nm.maxl - ln));
        int32_t group = -1;
        for (int64_t q = 0; q < nq; ++q) {
            const int qd[3] = {int(q % N1), int((q / N1) % N1), int(q / (N1 * N1))};
            double x[3], xi[3];
            for (int d = 0; d < 3; ++d) x[d] = nm.leaf[4 * e + 1 + d] + gp(qd[d]) * s;
            const double zn = nm.leaf[4 * e + 3] * nm.unit[2] + gp(qd[2]) * (s * nm.unit[2]);
            int32_t src;
            if (grow && x[2] > (double)om.top) {
                src = (ztop_new - zn <= c->powder_depth) ? -1 : -2;
            } else {
                const int32_t eo = oct_locate(om, x, xi);
                if (eo < 0) return fail(c, PBF_EMESH, "new point outside the old mesh");
                if (grow && om.leaf[4 * eo] > ln) {  // coarsened parent: the old children's points
                    if (group < 0) {
                        const int64_t h = (int64_t)1 << (om.maxl - ln - 1);
                        for (int k = 0; k < 8; ++k) {
                            const int32_t f = om.leaf_map.find(
                                ((uint64_t)(nm.leaf[4 * e + 1] + (k & 1) * h)) |
                                ((uint64_t)(nm.leaf[4 * e + 2] + ((k >> 1) & 1) * h) << 20) |
                                ((uint64_t)(nm.leaf[4 * e + 3] + ((k >> 2) & 1) * h) << 40) | ((uint64_t)(ln + 1) << 60));
                            if (f < 0 || om.cell_hist[f] < 0) return fail(c, PBF_EMESH, "coarsened leaf without its children");
                            for (int64_t qo = 0; qo < nq; ++qo)
                                c->pending.grp_idx.push_back((int32_t)(qo * om.n_hist_cells + om.cell_hist[f]));
                        }
                        c->pending.grp_start.push_back((int32_t)c->pending.grp_idx.size());
                        group = (int32_t)c->pending.grp_start.size() - 2;
                    }
                    src = -3 - group;
                } else {
                    int qo[3];
                    for (int d = 0; d < 3; ++d) {
                        qo[d] = 0;
                        for (int j = 1; j <= P; ++j)
                            if (std::fabs(xi[d] - gp(j)) < std::fabs(xi[d] - gp(qo[d]))) qo[d] = j;
                    }
                    const double so = (double)(1LL << (om.maxl - om.leaf[4 * eo]));
                    const double zo = om.leaf[4 * eo + 3] * om.unit[2] + gp(qo[2]) * (so * om.unit[2]);
                    if ((grow || ztop_old - zo <= c->powder_depth) && om.cell_hist[eo] >= 0)
                        src = (int32_t)((qo[0] + N1 * (qo[1] + N1 * qo[2])) * om.n_hist_cells + om.cell_hist[eo]);
                    else
                        src = (ztop_new - zn <= c->powder_depth) ? -1 : -2;
                }
            }
            c->pending.src[q * nm.n_hist_cells + hc] = src;
        }
    }
    std::swap(c->oct, nm);  // size the workspace of the new mesh
    size_t b = 0;
    pbf_status st = pbf_workspace_bytes(c, &b);
    std::swap(c->oct, nm);
    if (st) return st;
    b += align256(4 * (size_t)nm.n_dofs) + align256(24 * (size_t)nm.n_dofs) + align256(4 * c->pending.src.size()) +
         align256(4 * c->pending.grp_start.size()) + align256(4 * c->pending.grp_idx.size());
    if (new_n_dofs) *new_n_dofs = nm.n_dofs;
    if (new_n_hist_qp) *new_n_hist_qp = (int64_t)c->pending.src.size();
    c->pending.mesh = std::move(nm);
    c->pending.ready = true;
    *bytes = b;
    return PBF_OK;
}

pbf_status pbf_octree_remesh_bytes(pbf_ctx *c, int64_t n_leaves, const int32_t *leaves, size_t *bytes,
                                   int64_t *new_n_dofs, int64_t *new_n_hist_qp)
{
    if (!c || !leaves || !bytes) return fail(c, PBF_EINVAL, "NULL argument");
    if (!c->octree) return fail(c, PBF_ESTATE, "no octree mesh");
    pbf_status st = check_bound(c);
    if (st) return st;
    return prepare_remesh(c, n_leaves, leaves, c->oct.top, bytes, new_n_dofs, new_n_hist_qp);
}

pbf_status pbf_octree_grow_bytes(pbf_ctx *c, int64_t new_top, int64_t n_leaves, const int32_t *leaves, size_t *bytes,
                                 int64_t *new_n_dofs, int64_t *new_n_hist_qp)
{
    if (!c || !leaves || !bytes) return fail(c, PBF_EINVAL, "NULL argument");
    if (!c->octree || !c->oct.growing) return fail(c, PBF_ESTATE, "no growing octree (pbf_mesh_octree_growing)");
    pbf_status st = check_bound(c);
    if (st) return st;
    if (new_top < c->oct.top) return fail(c, PBF_EINVAL, "the active top cannot move down");
    return prepare_remesh(c, n_leaves, leaves, new_top, bytes, new_n_dofs, new_n_hist_qp);
}

pbf_status pbf_octree_remesh(pbf_ctx *c, void *workspace, size_t bytes, const double *T_old, const double *rc_old,
                             double *T_new, double *rc_new, void *stream)
{
    if (!c) return fail(nullptr, PBF_EINVAL, "ctx is NULL");
    if (!c->octree || !c->pending.ready) return fail(c, PBF_ESTATE, "call pbf_octree_remesh_bytes first");
    pbf_status st = check_bound(c);
    if (st) return st;
    if (!T_old || !T_new) return fail(c, PBF_EINVAL, "NULL temperature array");
    if (n_hist_qp(c) > 0 && !rc_old) return fail(c, PBF_EINVAL, "rc_old is NULL but the old mesh has history");
    if (c->pending.mesh.n_hist_cells > 0 && !rc_new)
        return fail(c, PBF_EINVAL, "rc_new is NULL but the new mesh has history");
    hipStream_t s = (hipStream_t)stream;
    const OctDev old = c->od;       // old tables stay valid until this call returns
    const int64_t old_hq = n_hist_qp(c);
    OctMesh old_mesh = std::move(c->oct);
    c->oct = std::move(c->pending.mesh);
    size_t need = 0;
    st = pbf_workspace_bytes(c, &need);
    const size_t N = (size_t)c->oct.n_dofs;
    const size_t total = need + align256(4 * N) + align256(24 * N) + align256(4 * c->pending.src.size()) +
                         align256(4 * c->pending.grp_start.size()) + align256(4 * c->pending.grp_idx.size());
    if (!st && bytes < total) st = fail(c, PBF_ENOMEM, "workspace too small: %zu < %zu bytes", bytes, total);
    if (st) {  // keep the old mesh and binding
        c->pending.mesh = std::move(c->oct);
        c->oct = std::move(old_mesh);
        return st;
    }
    c->pending.ready = false;
    if ((st = pbf_bind_device(c, workspace, bytes, stream))) {
        c->bound = false;
        return st;
    }
    char *p = (char *)workspace + need;
    int32_t *d_cell = (int32_t *)p;
    p += align256(4 * N);
    double *d_xi = (double *)p;
    p += align256(24 * N);
    int32_t *d_src = (int32_t *)p;
    p += align256(4 * c->pending.src.size());
    int32_t *d_gs = (int32_t *)p;
    p += align256(4 * c->pending.grp_start.size());
    int32_t *d_gi = (int32_t *)p;
    PBF_HIP(c, hipMemcpyAsync(d_cell, c->pending.cell.data(), 4 * N, hipMemcpyHostToDevice, s));
    PBF_HIP(c, hipMemcpyAsync(d_xi, c->pending.xi.data(), 24 * N, hipMemcpyHostToDevice, s));
    if (!c->pending.src.empty())
        PBF_HIP(c, hipMemcpyAsync(d_src, c->pending.src.data(), 4 * c->pending.src.size(), hipMemcpyHostToDevice, s));
    PBF_HIP(c, hipMemcpyAsync(d_gs, c->pending.grp_start.data(), 4 * c->pending.grp_start.size(), hipMemcpyHostToDevice, s));
    if (!c->pending.grp_idx.empty())
        PBF_HIP(c, hipMemcpyAsync(d_gi, c->pending.grp_idx.data(), 4 * c->pending.grp_idx.size(), hipMemcpyHostToDevice, s));
    PBF_HIP(c, launch_oct_transfer(c->degree, old, T_old, d_cell, d_xi, (int64_t)N, T_new, c->T_init,
                                   old_hq > 0 ? rc_old : nullptr, d_src, (int64_t)c->pending.src.size(), d_gs, d_gi,
                                   rc_new, s));
    PBF_HIP(c, hipStreamSynchronize(s));
    c->pending.cell.clear();
    c->pending.xi.clear();
    c->pending.src.clear();
    c->pending.grp_start.clear();
    c->pending.grp_idx.clear();
    return PBF_OK;
}

pbf_status pbf_timing_begin(pbf_ctx *c, int max_steps, int every)
{
    if (!c) return fail(nullptr, PBF_EINVAL, "ctx is NULL");
    if (max_steps < 1 || max_steps > (1 << 22)) return fail(c, PBF_EINVAL, "max_steps out of range");
    if (every < 1) return fail(c, PBF_EINVAL, "every must be >= 1");
    c->timing_every = every;
    c->timing_seen = 0;
    for (hipEvent_t e : c->tev) (void)hipEventDestroy(e);
    c->tev.assign((size_t)max_steps * 4, nullptr);
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
    const size_t n = c->tev_used / 4;
    if (n > 0) PBF_HIP(c, hipEventSynchronize(c->tev[c->tev_used - 1]));
    for (size_t k = 0; k < n; ++k) {
        float t1 = 0.f, t2 = 0.f;
        PBF_HIP(c, hipEventElapsedTime(&t1, c->tev[4 * k], c->tev[4 * k + 1]));
        PBF_HIP(c, hipEventElapsedTime(&t2, c->tev[4 * k + 2], c->tev[4 * k + 3]));
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
