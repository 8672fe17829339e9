// Host runtime behind the C ABI of include/lbm_ms.h: handle state, workspace layout, the pore-space
// clean-up and the fluid index map, the physical-to-lattice conversion, the stepping loop and the
// reductions.  Every per-node computation of the method runs in the HIP kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "lbm_ms.h"
#include "lbm_ms_kernels.hpp"

using namespace lbmms;

namespace {

constexpr double R_GAS = 8.3145;    // J / (mol K)
constexpr double FARADAY = 96485.0; // C / mol (Eq. 39)
constexpr int RED_BLOCKS = 1024;    // per-block partials of the reductions
constexpr uint64_t STATE_MAGIC = 0x334d534c42304c32ull;

struct Layout {
    size_t f[2], xn[2], idx, snap, field, part, prof, flags, scal, inst, tiles, ent, total;
    size_t tile_cap, ent_cap;
    size_t g[2], u[2], xa, vox;  // advective coupling: velocity model, node velocities, X and
                                 // voxel per compact node
    size_t c3off, c3pos;    // 3D fluid-compacted columns: plane offsets, in-column positions
};

int q_of(int lattice)
{
    return lattice == LBM_MS_D2Q9 ? 9 : lattice == LBM_MS_D2Q5 ? 5 : lattice == LBM_MS_D3Q7 ? 7 : 19;
}
bool known_lattice(int lattice)
{
    return lattice == LBM_MS_D2Q9 || lattice == LBM_MS_D3Q19 || lattice == LBM_MS_D2Q5 ||
           lattice == LBM_MS_D3Q7;
}
bool is_2d(int lattice) { return lattice == LBM_MS_D2Q9 || lattice == LBM_MS_D2Q5; }

size_t elem_bytes(int prec)
{
    switch (prec) {
    case LBM_MS_FP64: return 8;
    case LBM_MS_FP32: return 4;
    default: return 2;
    }
}

// Bounds of the 2D work lists for any tile height TY >= 4: a 64 x TY tile splits into at most two
// parts (64 TY nodes, 32 TY lanes); own entries total at most nx ny; each part lists at most
// (64 + 2)(TY + 2) halo entries, which is largest per node at TY = 4.
void tile_caps(int nx, int ny, size_t* tiles, size_t* ents)
{
    const size_t t4 = (size_t)((nx + 63) / 64) * (size_t)((ny + 3) / 4);
    *tiles = 2 * t4;
    *ents = (size_t)nx * ny + 2 * t4 * 66 * 6 + 4096;
}

bool node_shift(const lbm_ms_params& p)
{
    return p.precision != LBM_MS_FP64 && p.shift_mode == LBM_MS_SHIFT_NODE;
}

// the 3D fluid-compacted columns (launch shapes with tile_y 12 and 16) are built for global-shift
// storage in 32 or 16 bits
bool compacted3d(int lattice, int precision, int shift_mode)
{
    return !is_2d(lattice) && precision != LBM_MS_FP64 && shift_mode == LBM_MS_SHIFT_GLOBAL;
}
bool compacted3d(const lbm_ms_params& p) { return compacted3d(p.lattice, p.precision, p.shift_mode); }
bool compacted_ty(int ty) { return ty == 12 || ty == 16; }

// Visit the voxels of the 3D column plane with origin (x0, y0) and ylen rows in the order its
// fluid nodes are numbered: the two edge lines x = x0 and x = x0 + 63 first (y increasing),
// then the rows between in raster order.
constexpr int COL_X = 64, COL_Y = 16;
template <class Visit>
void column_plane_order(int nx, int ny, int x0, int y0, int ylen, Visit&& visit)
{
    const int x1 = std::min(x0 + COL_X, nx) - 1;  // last column of the box, or x0 + 63
    for (int y = y0; y < y0 + ylen && y < ny; ++y) visit(x0, y);
    if (x1 > x0)
        for (int y = y0; y < y0 + ylen && y < ny; ++y) visit(x1, y);
    for (int y = y0; y < y0 + ylen && y < ny; ++y)
        for (int x = x0 + 1; x < x1; ++x) visit(x, y);
}

// Plane lists of the fluid-compacted 3D columns: for column c = bx + tiles_x by (64 x ty voxels)
// and plane z, the in-column positions lx + 64 ly of its fluid voxels, in the order the fluid
// nodes are numbered (column_plane_order), are pos[off[c nz + z], off[c nz + z + 1]); off has
// tiles_x tiles_y nz + 1 entries.
void build_cols_3d(int nx, int ny, int nz, int ty, const std::vector<uint8_t>& mask,
                   std::vector<uint32_t>& off, std::vector<uint16_t>& pos)
{
    const int tx = (nx + 63) / 64, tyn = (ny + ty - 1) / ty;
    off.assign((size_t)tx * tyn * nz + 1, 0);
    pos.clear();
    for (int by = 0; by < tyn; ++by)
        for (int bx = 0; bx < tx; ++bx) {
            const size_t c = (size_t)bx + (size_t)tx * by;
            for (int z = 0; z < nz; ++z) {
                off[c * nz + z] = (uint32_t)pos.size();
                column_plane_order(nx, ny, bx * 64, by * ty, ty, [&](int x, int y) {
                    const size_t n = ((size_t)z * ny + y) * nx + x;
                    if (!mask[n]) pos.push_back((uint16_t)((x - bx * 64) + 64 * (y - by * ty)));
                });
            }
        }
    off.back() = (uint32_t)pos.size();
}

bool valid_params(const lbm_ms_params* p, std::string* why)
{
    auto fail = [&](const char* m) { if (why) *why = m; return false; };
    if (!p) return fail("params is NULL");
    if (!known_lattice(p->lattice)) return fail("unknown lattice");
    if (p->nx < 2 || p->ny < 1 || p->nz < 1) return fail("need nx >= 2, ny >= 1, nz >= 1");
    if (is_2d(p->lattice) && p->nz != 1) return fail("the 2D lattices need nz == 1");
    const long long N = (long long)p->nx * p->ny * p->nz;
    // the kernels address the index map with 32-bit byte offsets from its base
    if (N > (1ll << 30)) return fail("domain too large (more than 2^30 voxels)");
    if (p->precision < LBM_MS_FP64 || p->precision > LBM_MS_BF16) return fail("unknown precision");
    if (p->shift_mode != LBM_MS_SHIFT_GLOBAL && p->shift_mode != LBM_MS_SHIFT_NODE)
        return fail("unknown shift mode");
    if (p->ms_mode != LBM_MS_LOCAL_FLUX && p->ms_mode != LBM_MS_STOICH) return fail("unknown ms_mode");
    if (p->inlet_mode != LBM_MS_INLET_DIRICHLET && p->inlet_mode != LBM_MS_INLET_WALL)
        return fail("unknown inlet mode");
    if (p->collision != LBM_MS_BGK && p->collision != LBM_MS_TRT) return fail("unknown collision");
    if (!std::isfinite(p->trt_lambda)) return fail("trt_lambda must be finite");
    if (!(p->T > 0) || !(p->p > 0) || !(p->dx > 0)) return fail("T, p, dx must be positive");
    if (!(p->tau_ref > 0.5)) return fail("tau_ref must exceed 1/2");
    const double d12 = p->D[1], d13 = p->D[2], d23 = p->D[5];
    if (!(d12 > 0) || !(d13 > 0) || !(d23 > 0)) return fail("binary diffusivities must be positive");
    if (p->D[3] != d12 || p->D[6] != d13 || p->D[7] != d23) return fail("D must be symmetric");
    if (p->advection != 0 && p->advection != 1) return fail("advection must be 0 or 1");
    if (!p->advection) {
        if (p->nu[2] != 0 || p->nu[0] == 0 || p->nu[0] != -p->nu[1])
            return fail("need nu1 = -nu2 != 0 and nu3 = 0 (equimolar counter-diffusion); a "
                        "reaction that changes the number of moles needs advection = 1");
    } else {
        if (p->nu[2] != 0 || p->nu[0] == 0 || p->nu[1] == 0)
            return fail("advection: need nu1 != 0, nu2 != 0, nu3 = 0");
        // the 1D steady flux ratios (-nu_j - X_j Nt) / (-nu_i - X_i Nt) must stay finite for
        // X in [0, 1]: -nu_i and -nu_i - Nt nonzero and of one sign
        const double nt = -(double)(p->nu[0] + p->nu[1]);
        for (int i = 0; i < 2; ++i) {
            const double a0 = -(double)p->nu[i], a1 = a0 - nt;
            if (!(a0 * a1 > 0)) return fail("advection: these nu make a 1D flux ratio vanish");
        }
        if (p->precision != LBM_MS_FP64 && p->precision != LBM_MS_FP32)
            return fail("advection: FP64 or FP32 storage");
        if (p->shift_mode != LBM_MS_SHIFT_GLOBAL) return fail("advection: global storage only");
        if (p->collision != LBM_MS_BGK) return fail("advection: BGK collision only");
        if (p->inlet_mode != LBM_MS_INLET_DIRICHLET) return fail("advection: Dirichlet inlet only");
        if (!(p->tau_flow <= 0 || p->tau_flow > 0.5)) return fail("advection: tau_flow must exceed 1/2");
    }
    if (p->n_electrons <= 0) return fail("n_electrons must be positive");
    return true;
}

// Elements between consecutive (species, link) population planes for n stored nodes: n rounded up
// to 64 elements plus an odd multiple of 64, so the 2Q planes of one node do not sit a power of
// two apart.
long long plane_pitch(long long n)
{
    return ((n + 63) / 64) * 64 + 192;
}

Layout layout(const lbm_ms_params& p)
{
    Layout L{};
    const size_t N = (size_t)p.nx * p.ny * p.nz;
    const int q = q_of(p.lattice);
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off += (bytes + 255) & ~(size_t)255; return o; };
    // sized for the all-fluid box; the fluid count is known only at set_geometry
    const size_t fb = 2ull * q * (size_t)plane_pitch((long long)N) * elem_bytes(p.precision);
    L.f[0] = take(fb);
    L.f[1] = take(fb);
    const size_t xb = node_shift(p) ? 2ull * N * sizeof(double) : 0;
    L.xn[0] = take(xb);
    L.xn[1] = take(xb);
    L.idx = take(N * sizeof(int32_t));
    L.snap = take(2ull * N * sizeof(double));
    L.field = take(3ull * N * sizeof(double));
    L.part = take((size_t)RED_BLOCKS * 8 * sizeof(double));
    L.prof = take(2ull * p.nx * sizeof(double));
    L.flags = take(64);
    L.scal = take(64 * sizeof(double));
    // 2D work lists: tiles of 64 x TY (TY >= 4) and their entries
    L.tile_cap = 0;
    L.ent_cap = 0;
    if (is_2d(p.lattice)) tile_caps(p.nx, p.ny, &L.tile_cap, &L.ent_cap);
    L.inst = take(2 * sizeof(StepArgs));
    L.tiles = take(L.tile_cap * 2 * sizeof(int4));
    L.ent = take(L.ent_cap * sizeof(uint32_t));
    L.c3off = L.c3pos = 0;
    if (compacted3d(p)) {
        const size_t cols = (size_t)((p.nx + 63) / 64) * (size_t)((p.ny + 11) / 12);  // most at ty 12
        L.c3off = take((cols * (size_t)p.nz + 1) * sizeof(uint32_t));
        L.c3pos = take(N * sizeof(uint16_t));
    }
    if (p.advection) {
        const size_t gb = (size_t)q * (size_t)plane_pitch((long long)N) * elem_bytes(p.precision);
        L.g[0] = take(gb);
        L.g[1] = take(gb);
        L.u[0] = take(3ull * N * sizeof(double));
        L.u[1] = take(3ull * N * sizeof(double));
        L.xa = take(2ull * N * sizeof(double));
        L.vox = take(N * sizeof(int32_t));
    }
    L.total = off;
    return L;
}

void build_tiles_2d(int nx, int ny, int ty, int rows, const std::vector<uint8_t>& solid, int instance,
                    uint32_t ent_base, std::vector<int4>& tiles, std::vector<uint32_t>& ent);
bool tiles_in_bounds(const std::vector<int4>& tiles, const std::vector<uint32_t>& ent, int ty, int rows);

}  // namespace

struct lbm_ms_s {
    lbm_ms_params p{};
    hipStream_t stream = nullptr;
    Layout L{};
    char* ws = nullptr;
    int q = 9;
    long long N = 0;
    long long P = 0;
    int cur = 0;
    // host state
    std::vector<uint8_t> mask;
    long long n_fluid = 0, n_open = 0;
    double dt = 0, Ct = 0, Dl[9] = {0}, Q[2] = {0, 0}, Qs[2] = {0, 0}, Xin[3] = {0, 0, 0};
    double j = 0, eps = 0, tau_min = 0, tau_max = 0;
    double S[2] = {0, 0};   // volumetric source per fluid node and step of the columns x >= src_x0
    int src_x0 = 1 << 30;   // no source
    long long n_src = 0;
    bool geom = false, bc = false, ready = false;
    long long steps = 0, snap_step = 0;
    int ty = 0, cz = 0;
    int ntiles = 0;
    int c3_ty = 0;  // tile height the 3D column lists in the workspace were built for (0: none)
    double* pinned = nullptr;
    std::string err;

    int fail(int code, const char* fmt, ...)
    {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof(buf), fmt, ap);
        va_end(ap);
        err = buf;
        return code;
    }
    int hip(hipError_t e, const char* what)
    {
        if (e == hipSuccess) return LBM_MS_OK;
        return fail(LBM_MS_E_HIP, "%s: %s", what, hipGetErrorString(e));
    }
    void* at(size_t off) { return ws + off; }
    int prec() const { return p.precision; }
    int ns() const { return node_shift(p) ? 1 : 0; }

    StepArgs args(int in_buf) const
    {
        StepArgs a{};
        a.fin = ws + L.f[in_buf];
        a.fout = ws + L.f[1 - in_buf];
        a.xin = node_shift(p) ? reinterpret_cast<const double*>(ws + L.xn[in_buf]) : nullptr;
        a.xout = node_shift(p) ? reinterpret_cast<double*>(ws + L.xn[1 - in_buf]) : nullptr;
        a.idx = reinterpret_cast<const int*>(ws + L.idx);
        a.flags = reinterpret_cast<unsigned*>(ws + L.flags);
        a.N = N;
        a.NF = n_fluid;
        a.P = P;
        a.nx = p.nx;
        a.ny = p.ny;
        a.nz = p.nz;
        a.tiles_x = (p.nx + 63) / 64;
        a.tiles_y = (p.ny + ty - 1) / ty;
        a.chunks_z = !is_2d(p.lattice) ? (p.nz + cz - 1) / cz : 1;
        a.iD12 = 1.0 / Dl[1];
        a.iD13 = 1.0 / Dl[2];
        a.iD23 = 1.0 / Dl[5];
        a.Xin0 = Xin[0];
        a.Xin1 = Xin[1];
        a.Q0 = Q[0];
        a.Q1 = Q[1];
        a.eps0 = eps * std::fabs((double)p.nu[0]);
        a.eps1 = eps * std::fabs((double)p.nu[1]);
        const double s0 = p.nu[0] > 0 ? -1.0 : 1.0, s1 = p.nu[1] > 0 ? -1.0 : 1.0;
        a.sgn12 = s0 * s1;
        a.rst21 = std::fabs((double)p.nu[1]) / std::fabs((double)p.nu[0]);
        a.rst12 = std::fabs((double)p.nu[0]) / std::fabs((double)p.nu[1]);
        a.c0 = Xin[0];
        a.c1 = Xin[1];
        a.om_lo = 1.0 / tau_max;
        a.om_hi = 1.0 / tau_min;
        a.ms_mode = p.ms_mode;
        a.inlet_wall = p.inlet_mode == LBM_MS_INLET_WALL ? 1 : 0;
        a.S0 = S[0];
        a.S1 = S[1];
        a.src_x0 = src_x0 < p.nx ? src_x0 : p.nx;
        a.trt = p.collision == LBM_MS_TRT ? 1 : 0;
        a.trt_lambda = p.trt_lambda > 0 ? p.trt_lambda : 0.25;
        return a;
    }
    // advective coupling: the velocity model's buffers of a step that reads parity in_buf
    AdvArgs adv_args(int in_buf) const
    {
        AdvArgs v{};
        v.gin = ws + L.g[in_buf];
        v.gout = ws + L.g[1 - in_buf];
        v.xc = reinterpret_cast<const double*>(ws + L.xa);
        v.uin = reinterpret_cast<const double*>(ws + L.u[in_buf]);
        v.uout = reinterpret_cast<double*>(ws + L.u[1 - in_buf]);
        v.Qt = Q[0] + Q[1];
        v.om_flow = 1.0 / (p.tau_flow > 0 ? p.tau_flow : 1.0);
        v.nh0 = -(double)p.nu[0];
        v.nh1 = -(double)p.nu[1];
        v.nh2 = -(double)p.nu[2];
        v.nht = v.nh0 + v.nh1 + v.nh2;
        v.eps2 = eps * eps;
        v.vox = p.advection ? reinterpret_cast<const int*>(ws + L.vox) : nullptr;
        return v;
    }
    int nblocks_step() const
    {
        const long long tx = (p.nx + 63) / 64, tyy = (p.ny + ty - 1) / ty;
        const long long tz = !is_2d(p.lattice) ? (p.nz + cz - 1) / cz : 1;
        return (int)(tx * tyy * tz);
    }
    int sync() { return hip(hipStreamSynchronize(stream), "hipStreamSynchronize"); }

    // instance table of both step parities (read by the 2D work-list kernel)
    int upload_tables()
    {
        StepArgs t[2] = {args(0), args(1)};
        int rc = sync();
        if (rc) return rc;
        std::memcpy(pinned + 64, t, sizeof(t));
        rc = hip(hipMemcpyAsync(ws + L.inst, pinned + 64, sizeof(t), hipMemcpyHostToDevice, stream),
                 "instance table upload");
        if (rc) return rc;
        return sync();
    }

    int upload_tiles()
    {
        if (!geom) return LBM_MS_OK;
        if (!is_2d(p.lattice)) {
            if (!compacted_ty(ty)) return LBM_MS_OK;
            std::vector<uint32_t> off;
            std::vector<uint16_t> pos;
            build_cols_3d(p.nx, p.ny, p.nz, ty, mask, off, pos);
            const size_t cap_off = (size_t)((p.nx + 63) / 64) * (size_t)((p.ny + 11) / 12) * p.nz + 1;
            if (!compacted3d(p) || off.size() > cap_off || pos.size() != (size_t)n_fluid)
                return fail(LBM_MS_E_ARG, "compacted column lists do not fit this handle");
            int rc = hip(hipMemcpyAsync(ws + L.c3off, off.data(), off.size() * sizeof(uint32_t),
                                        hipMemcpyHostToDevice, stream), "column list upload");
            if (rc) return rc;
            rc = hip(hipMemcpyAsync(ws + L.c3pos, pos.data(), pos.size() * sizeof(uint16_t),
                                    hipMemcpyHostToDevice, stream), "column list upload");
            if (rc) return rc;
            c3_ty = ty;
            return sync();
        }
        std::vector<int4> tl;
        std::vector<uint32_t> en;
        build_tiles_2d(p.nx, p.ny, ty, cz, mask, 0, 0, tl, en);
        if (tl.size() / 2 > L.tile_cap || en.size() > L.ent_cap)
            return fail(LBM_MS_E_NOMEM, "work list exceeds its workspace share");
        if (!tiles_in_bounds(tl, en, ty, cz)) return fail(LBM_MS_E_ARG, "work list out of bounds");
        int rc = hip(hipMemcpyAsync(ws + L.tiles, tl.data(), tl.size() * sizeof(int4),
                                    hipMemcpyHostToDevice, stream), "tile upload");
        if (rc) return rc;
        rc = hip(hipMemcpyAsync(ws + L.ent, en.data(), en.size() * sizeof(uint32_t),
                                hipMemcpyHostToDevice, stream), "entry upload");
        if (rc) return rc;
        ntiles = (int)(tl.size() / 2);
        return sync();
    }
};

// ---------------------------------------------------------------------------------------------
// pore-space clean-up and the fluid index map (host)
// ---------------------------------------------------------------------------------------------
namespace {

struct HostLattice {
    int q;
    int e[19][3];
};

HostLattice host_lattice(int lattice)
{
    HostLattice H{};
    H.q = q_of(lattice);
    for (int k = 0; k < H.q; ++k) {
        if (lattice == LBM_MS_D2Q9) {
            H.e[k][0] = D2Q9::ex[k];
            H.e[k][1] = D2Q9::ey[k];
            H.e[k][2] = 0;
        } else if (lattice == LBM_MS_D2Q5) {
            H.e[k][0] = D2Q5::ex[k];
            H.e[k][1] = D2Q5::ey[k];
            H.e[k][2] = 0;
        } else if (lattice == LBM_MS_D3Q7) {
            H.e[k][0] = D3Q7::ex[k];
            H.e[k][1] = D3Q7::ey[k];
            H.e[k][2] = D3Q7::ez[k];
        } else {
            H.e[k][0] = D3Q19::ex[k];
            H.e[k][1] = D3Q19::ey[k];
            H.e[k][2] = D3Q19::ez[k];
        }
    }
    return H;
}

// Breadth-first search over lattice links from every fluid node of the inlet column; fluid that
// is not reached becomes solid.  Returns the number of reached outlet-column nodes.
long long clean_pores(const lbm_ms_params& p, std::vector<uint8_t>& solid)
{
    const HostLattice H = host_lattice(p.lattice);
    const int nx = p.nx, ny = p.ny, nz = p.nz;
    const long long N = (long long)nx * ny * nz;
    std::vector<uint8_t> seen(N, 0);
    std::vector<long long> queue;
    queue.reserve(N / 4 + 16);
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y) {
            const long long n = ((long long)z * ny + y) * nx;
            if (!solid[n]) { seen[n] = 1; queue.push_back(n); }
        }
    for (size_t head = 0; head < queue.size(); ++head) {
        const long long n = queue[head];
        const int x = (int)(n % nx);
        const int y = (int)((n / nx) % ny);
        const int z = (int)(n / ((long long)nx * ny));
        for (int k = 1; k < H.q; ++k) {
            const int xx = x + H.e[k][0];
            if (xx < 0 || xx >= nx) continue;
            const int yy = (y + H.e[k][1] + ny) % ny;
            const int zz = (z + H.e[k][2] + nz) % nz;
            const long long m = ((long long)zz * ny + yy) * nx + xx;
            if (!solid[m] && !seen[m]) { seen[m] = 1; queue.push_back(m); }
        }
    }
    long long open = 0;
    for (long long n = 0; n < N; ++n) {
        solid[n] = seen[n] ? 0 : 1;
        if (seen[n] && (n % nx) == nx - 1) ++open;
    }
    return open;
}

// Fluid nodes of a 2D box are numbered in raster order (x fastest).  A 3D box is numbered by
// Fluid-node numbering.  2D: strips 64 voxels wide (the width of a work-list tile), strip by
// strip, each in raster order, so that a tile's nodes are one contiguous run of each link's
// array and no cache line is shared with the tile beside it in x (with raster order over the
// whole box each tile row was a short run whose end lines the neighbouring tile, processed at
// another time, read and wrote again).  3D: columns of 64 x 16 voxels (x-column fastest, then
// y), each column plane by plane: the nodes a marching workgroup pulls in one plane then sit
// together in memory instead of sharing cache lines with the columns beside it, which march out
// of step.  Within a column's plane come first its two edge lines x = x0 and x = x0 + 63 (y
// increasing; the voxels a neighbouring column reads as its side halo, now one short run each),
// then the rows between in raster order.  Solid voxels map to -1.
long long build_index(const std::vector<uint8_t>& solid, int nx, int ny, int nz,
                      std::vector<int32_t>& idx)
{
    idx.assign(solid.size(), -1);
    long long k = 0;
    if (nz == 1) {
        for (int x0 = 0; x0 < nx; x0 += COL_X)
            for (int y = 0; y < ny; ++y)
                for (int x = x0; x < std::min(x0 + COL_X, nx); ++x)
                    if (!solid[(size_t)y * nx + x]) idx[(size_t)y * nx + x] = (int32_t)k++;
        return k;
    }
    for (int y0 = 0; y0 < ny; y0 += COL_Y)
        for (int x0 = 0; x0 < nx; x0 += COL_X)
            for (int z = 0; z < nz; ++z)
                column_plane_order(nx, ny, x0, y0, COL_Y, [&](int x, int y) {
                    const size_t n = ((size_t)z * ny + y) * nx + x;
                    if (!solid[n]) idx[n] = (int32_t)k++;
                });
    return k;
}

// 2D work list: per tile the fluid nodes it updates (own) and the other fluid nodes whose moments
// its gradients read (halo: axis neighbours of own nodes, including rows past the end of the box,
// which hold the periodic image).  Entries are moment-tile coordinates (cx, cy) =
// (x - x0 + 1, y - y0 + 1) packed as cy << 8 | cx.  Tiles without fluid are dropped.  Entry
// offsets are ent_base + the position in ent (several instances may append to one ent).
//  - rows == 0: fixed 64 x ty tiles; a tile with more than 32 ty fluid nodes is split into parts.
//  - rows > 0: packed tiles: each 64-wide strip is cut into tiles of consecutive rows, a tile
//    growing until one more row would exceed 32 ty fluid nodes or `rows` rows, so no tile splits
//    and more lanes hold a node (at least 4 rows per tile for 32 ty >= 256).
void build_tiles_2d(int nx, int ny, int ty, int rows, const std::vector<uint8_t>& solid, int instance,
                    uint32_t ent_base, std::vector<int4>& tiles, std::vector<uint32_t>& ent)
{
    const int TX = 64;
    const int RT = rows > 0 ? rows : ty;  // rows of the moment tile
    const size_t lanes = (size_t)32 * ty;  // workgroup size: one own node per lane
    auto fluid = [&](int x, int y) { return !solid[(size_t)y * nx + x]; };
    std::vector<uint8_t> mark((TX + 2) * (RT + 2));
    std::vector<uint32_t> own;
    static const int dxy[4][2] = {{1, 0}, {-1, 0}, {0, 1}, {0, -1}};
    // own nodes [start, stop) of the tile at (x0, y0) and their halo
    auto emit = [&](int x0, int y0, size_t start, size_t stop) {
        std::fill(mark.begin(), mark.end(), 0);
        const uint32_t own_off = ent_base + (uint32_t)ent.size();
        for (size_t e = start; e < stop; ++e) {
            ent.push_back(own[e]);
            mark[(own[e] >> 8) * (TX + 2) + (own[e] & 255u)] = 1;
        }
        const uint32_t halo_off = ent_base + (uint32_t)ent.size();
        for (size_t e = start; e < stop; ++e) {
            const int cx = own[e] & 255u, cy = own[e] >> 8;
            for (auto& d : dxy) {
                const int hx = cx + d[0], hy = cy + d[1];
                const int gx = x0 + hx - 1;
                if (gx < 0 || gx >= nx) continue;
                const int gy = ((y0 + hy - 1) % ny + ny) % ny;
                if (!fluid(gx, gy) || mark[hy * (TX + 2) + hx]) continue;
                mark[hy * (TX + 2) + hx] = 2;
                ent.push_back((uint32_t)(hy << 8 | hx));
            }
        }
        const uint32_t halo_cnt = ent_base + (uint32_t)ent.size() - halo_off;
        tiles.push_back(make_int4(x0, y0, instance, 0));
        tiles.push_back(make_int4((int)own_off, (int)(stop - start), (int)halo_off, (int)halo_cnt));
    };
    auto row_nodes = [&](int x0, int y, int cy) {  // append row y of the strip as tile row cy
        for (int cx = 1; cx <= TX; ++cx) {
            const int x = x0 + cx - 1;
            if (x < nx && fluid(x, y)) own.push_back((uint32_t)(cy << 8 | cx));
        }
    };
    // Tiles are listed in row-band order (y0, then x0), so the tiles that run together on one XCD
    // span the box in x.  With fluid nodes numbered in 64-wide strips (build_index) a tile's
    // nodes are one run per link and its halo rows sit in the runs of the tiles above and below
    // it; listing the tiles strip by strip instead measured 1% slower.
    if (rows > 0) {
        const size_t first = tiles.size();
        for (int x0 = 0; x0 < nx; x0 += TX)
            for (int y0 = 0; y0 < ny;) {
                own.clear();
                int r = 0;
                while (r < rows && y0 + r < ny) {
                    const size_t before = own.size();
                    row_nodes(x0, y0 + r, r + 1);
                    if (own.size() > lanes) {  // this row does not fit: it starts the next tile
                        own.resize(before);
                        break;
                    }
                    ++r;
                }
                if (!own.empty()) emit(x0, y0, 0, own.size());
                y0 += r;
            }
        // each tile is two int4 records; order the pairs by (y0, x0)
        std::vector<std::pair<int4, int4>> pairs;
        for (size_t t = first; t + 1 < tiles.size(); t += 2) pairs.emplace_back(tiles[t], tiles[t + 1]);
        std::stable_sort(pairs.begin(), pairs.end(), [](const std::pair<int4, int4>& u, const std::pair<int4, int4>& v) {
            return u.first.y != v.first.y ? u.first.y < v.first.y : u.first.x < v.first.x;
        });
        tiles.resize(first);
        for (auto& pr : pairs) {
            tiles.push_back(pr.first);
            tiles.push_back(pr.second);
        }
        return;
    }
    for (int y0 = 0; y0 < ny; y0 += ty)
        for (int x0 = 0; x0 < nx; x0 += TX) {
            own.clear();
            for (int cy = 1; cy <= ty && y0 + cy - 1 < ny; ++cy) row_nodes(x0, y0 + cy - 1, cy);
            // parts of at most `lanes` own nodes (raster order, so a split runs along rows); each
            // part's halo: the fluid axis neighbours of its nodes outside the part, other parts
            // of the tile included
            for (size_t start = 0; start < own.size(); start += lanes)
                emit(x0, y0, start, std::min(own.size(), start + lanes));
        }
}

// Every tile's entry ranges lie inside the entry array and every entry inside the moment tile.
bool tiles_in_bounds(const std::vector<int4>& tiles, const std::vector<uint32_t>& ent, int ty, int rows)
{
    const size_t n_ent = ent.size();
    const uint32_t rt = (uint32_t)(rows > 0 ? rows : ty);  // rows of the moment tile
    for (size_t t = 0; t + 1 < tiles.size(); t += 2) {
        const int4 r = tiles[t + 1];
        if (r.x < 0 || r.y < 0 || r.z < 0 || r.w < 0) return false;
        if ((size_t)r.x + (size_t)r.y > n_ent || (size_t)r.z + (size_t)r.w > n_ent) return false;
        if (r.y > 32 * ty) return false;  // a lane holds at most one own node
        if (r.z != r.x + r.y) return false;  // halo entries follow the own entries
        for (int e = 0; e < r.y + r.w; ++e) {
            const uint32_t v = ent[e < r.y ? (size_t)r.x + e : (size_t)r.z + (e - r.y)];
            const uint32_t cx = v & 255u, cy = v >> 8;
            if (cx > 65u || cy > rt + 1u) return false;
            if (e < r.y && (cx < 1u || cx > 64u || cy < 1u || cy > rt)) return false;
        }
    }
    return true;
}

int default_tile_y(const lbm_ms_params& p)
{
    if (p.tile_y > 0) return p.tile_y;
    if (is_2d(p.lattice)) return p.ny >= 8 ? 8 : 4;
    // measured on a 256^3 porous block: D3Q19 FP64 runs best with the 256-lane tiles (its
    // 512-lane build spills), every other mode, D3Q7 included, with the 512-lane ones (D3Q7
    // with 16-bit storage is built for four waves per SIMD: BF16 0.339 ms against 0.369 ms on
    // 256-lane tiles)
    if (p.lattice == LBM_MS_D3Q7) return 8;
    // D3Q19 with global-shift 32- or 16-bit storage: the fluid-compacted 64 x 16 columns (FP32
    // 0.754 ms against 0.886 ms for 64 x 8 voxels per workgroup, BF16 0.624 against 0.807);
    // D3Q7 keeps 64 x 8 (0.368 ms against 0.396 ms compacted)
    if (compacted3d(p)) return 16;
    return p.precision == LBM_MS_FP64 ? 4 : 8;
}

int default_chunk_z(const lbm_ms_params& p)
{
    // 2D: the packed tiles' row limit.  Packed 64-wide tiles of up to 256 fluid nodes measured
    // faster than fixed 64 x 8 tiles on every 2D workload: more lanes hold a node and no tile
    // splits.  Best row limit on the 1024^2 slice: 9 for D2Q9 in every storage mode (FP32
    // 17.3 us; 12 rows 17.9, fixed 18.5), 12 for D2Q5 with global-shift or FP64 storage (FP32
    // 12.5 us; 10 rows 13.0, fixed 14.0) and 9 for D2Q5 with the NODE shift, whose staged
    // references make 12-row tiles slower than fixed ones (FP32 18.0 us; 12 rows 19.4, fixed 18.3).
    if (is_2d(p.lattice)) {
        if (p.chunk_z > 0) return p.chunk_z;
        if (default_tile_y(p) != 8) return 0;
        return (p.lattice == LBM_MS_D2Q5 && !node_shift(p)) ? 12 : 9;
    }
    if (p.chunk_z > 0) return p.chunk_z;
    if (compacted_ty(default_tile_y(p))) {
        // one workgroup per CU: the longest chunk (64, 32, 16 planes) that still gives every CU
        // a workgroup (256^3 D3Q19 FP32 with 64 x 16 columns: 0.754 / 0.787 / 0.795 ms)
        const int ty = default_tile_y(p);
        int dev = 0, cus = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0) {
            const long long cols = (long long)((p.nx + 63) / 64) * ((p.ny + ty - 1) / ty);
            for (int cz : {64, 32})
                if (cols * ((p.nz + cz - 1) / cz) >= (long long)cus) return cz;
        }
        return ty == 16 ? 16 : 32;
    }
    // Longer chunks spread each workgroup's prologue (five staged planes) over more planes, as
    // long as the grid still fills every resident workgroup slot: the largest of 128, 64 and 32
    // planes that does.  Measured on the 256^3 block with 512-lane tiles (32 -> 64 -> 128
    // planes): D3Q19 FP32 0.936 -> 0.898 -> 0.881 ms, BF16 0.845 -> 0.814 -> 0.797, FP32 NODE
    // 1.594 -> 1.519 -> 1.468; D3Q7 FP32 NODE 0.771 -> 0.757 -> 0.724.  D3Q7 FP32 holds two
    // workgroups per CU, so 128 planes (256 workgroups) leave half the slots empty: 0.371 ms at
    // 64 against 0.457 at 128.  FP64 (not measured beyond 32) keeps the rule below.
    const int ty = default_tile_y(p);
    if (ty == 8 && p.precision != LBM_MS_FP64) {
        int dev = 0, cus = 0;
        const int per_cu = step3d_resident_blocks(p.lattice, p.precision, node_shift(p) ? 1 : 0, ty);
        if (per_cu > 0 && hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0) {
            const long long cols = (long long)((p.nx + 63) / 64) * ((p.ny + ty - 1) / ty);
            for (int cz : {128, 64})
                if (cols * ((p.nz + cz - 1) / cz) >= (long long)per_cu * cus) return cz;
        }
    }
    return p.nz >= 128 ? 32 : 16;
}

bool tile_ok(int lattice, bool compacted, int ty, int cz)
{
    int tys[16], czs[16];
    const int n = tile_options(lattice, compacted, tys, czs, 16);
    for (int i = 0; i < n; ++i)
        if (tys[i] == ty && czs[i] == cz) return true;
    return false;
}

uint64_t param_hash(const lbm_ms_params& p, long long n_fluid)
{
    // FNV-1a over the fields that fix the state layout
    uint64_t h = 1469598103934665603ull;
    auto mix = [&](const void* d, size_t n) {
        const unsigned char* c = (const unsigned char*)d;
        for (size_t i = 0; i < n; ++i) { h ^= c[i]; h *= 1099511628211ull; }
    };
    mix(&p.lattice, sizeof(int)); mix(&p.nx, sizeof(int)); mix(&p.ny, sizeof(int));
    mix(&p.nz, sizeof(int)); mix(&p.precision, sizeof(int)); mix(&p.shift_mode, sizeof(int));
    mix(&n_fluid, sizeof(n_fluid));
    return h;
}

}  // namespace

// ---------------------------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------------------------
extern "C" {

namespace {
// Why the last create (or workspace query) on this thread failed: the calls that return no
// handle report through it (lbm_ms_last_error / lbm_ms_batch_last_error with NULL).
thread_local std::string g_create_err;
int create_fail(int code, const std::string& why)
{
    g_create_err = why;
    return code;
}
}  // namespace

size_t lbm_ms_workspace_bytes(const lbm_ms_params* params)
{
    std::string why;
    if (!valid_params(params, &why)) {
        g_create_err = "invalid parameters: " + why;
        return 0;
    }
    return layout(*params).total;
}

int lbm_ms_create(const lbm_ms_params* params, void* d_workspace, size_t bytes, lbm_ms_t* out)
{
    g_create_err.clear();
    if (!out) return create_fail(LBM_MS_E_ARG, "out is NULL");
    *out = nullptr;
    std::string why;
    if (!valid_params(params, &why)) return create_fail(LBM_MS_E_ARG, "invalid parameters: " + why);
    if (!d_workspace || ((uintptr_t)d_workspace & 255))
        return create_fail(LBM_MS_E_ARG, "workspace is NULL or not 256-byte aligned");
    const Layout L = layout(*params);
    if (bytes < L.total)
        return create_fail(LBM_MS_E_NOMEM, "workspace of " + std::to_string(bytes) + " bytes, " +
                                               std::to_string(L.total) + " needed");
    lbm_ms_s* h = new (std::nothrow) lbm_ms_s();
    if (!h) return create_fail(LBM_MS_E_NOMEM, "host allocation failed");
    h->p = *params;
    h->stream = (hipStream_t)params->stream;
    h->L = L;
    h->ws = (char*)d_workspace;
    h->q = q_of(params->lattice);
    h->N = (long long)params->nx * params->ny * params->nz;
    h->ty = default_tile_y(*params);
    h->cz = default_chunk_z(*params);
    if (!tile_ok(params->lattice, compacted3d(*params), h->ty, h->cz)) {
        delete h;
        return create_fail(LBM_MS_E_ARG, "tile shape not among lbm_ms_tile_options for this lattice");
    }
    h->tau_min = params->tau_min > 0 ? params->tau_min : 0.5 + 1e-9;
    h->tau_max = params->tau_max > 0 ? params->tau_max : 1e6;
    // lattice units: dt from tau_ref for the fastest pair (Eq. 25 with c_s^2 = 1/3)
    const double Dmax = std::max(params->D[1], std::max(params->D[2], params->D[5]));
    h->dt = (params->tau_ref - 0.5) * params->dx * params->dx / (3.0 * Dmax);
    for (int i = 0; i < 9; ++i) h->Dl[i] = params->D[i] * h->dt / (params->dx * params->dx);
    h->Ct = params->p / (R_GAS * params->T);
    if (hipHostMalloc((void**)&h->pinned, 4096) != hipSuccess) {
        delete h;
        return create_fail(LBM_MS_E_HIP, "hipHostMalloc of the pinned readback page failed");
    }
    // clear the flag words
    if (hipMemsetAsync(h->at(L.flags), 0, 64, h->stream) != hipSuccess) {
        hipHostFree(h->pinned);
        delete h;
        return create_fail(LBM_MS_E_HIP, "hipMemsetAsync of the flag words failed");
    }
    *out = h;
    return LBM_MS_OK;
}

void lbm_ms_destroy(lbm_ms_t h)
{
    if (!h) return;
    hipStreamSynchronize(h->stream);
    if (h->pinned) hipHostFree(h->pinned);
    delete h;
}

const char* lbm_ms_last_error(lbm_ms_t h)
{
    if (h) return h->err.c_str();
    return g_create_err.empty() ? "null handle" : g_create_err.c_str();
}

const char* lbm_ms_status_string(int s)
{
    switch (s) {
    case LBM_MS_OK: return "ok";
    case LBM_MS_E_ARG: return "invalid argument";
    case LBM_MS_E_STATE: return "call out of order";
    case LBM_MS_E_GEOM: return "outlet not connected to the inlet";
    case LBM_MS_E_HIP: return "HIP runtime error";
    case LBM_MS_E_DIVERGED: return "non-finite mole fraction";
    case LBM_MS_E_NOT_CONVERGED: return "not converged within max_steps";
    case LBM_MS_E_NEG_FRACTION: return "negative mole fraction (limiting current exceeded)";
    case LBM_MS_E_NOMEM: return "workspace too small or out of memory";
    case LBM_MS_E_TAU_CLAMP: return "relaxation time clamped";
    }
    return "unknown status";
}

int lbm_ms_lattice_info(int lattice, int* q, int* e, double* w)
{
    if (!known_lattice(lattice)) return LBM_MS_E_ARG;
    const int Q = q_of(lattice);
    if (q) *q = Q;
    auto put = [&](auto L) {
        using Lat = decltype(L);
        for (int k = 0; k < Q; ++k) {
            if (e) {
                e[3 * k + 0] = Lat::ex[k];
                e[3 * k + 1] = Lat::ey[k];
                e[3 * k + 2] = Lat::ez[k];
            }
            if (w) w[k] = Lat::w[k];
        }
    };
    if (lattice == LBM_MS_D2Q9) put(D2Q9{});
    else if (lattice == LBM_MS_D2Q5) put(D2Q5{});
    else if (lattice == LBM_MS_D3Q7) put(D3Q7{});
    else put(D3Q19{});
    return LBM_MS_OK;
}

int lbm_ms_tile_options(int lattice, int precision, int shift_mode, int* tile_y, int* chunk_z, int cap)
{
    if (!known_lattice(lattice)) return LBM_MS_E_ARG;
    return tile_options(lattice, compacted3d(lattice, precision, shift_mode), tile_y, chunk_z, cap);
}

int lbm_ms_set_tile(lbm_ms_t h, int tile_y, int chunk_z)
{
    if (!h) return LBM_MS_E_ARG;
    if (!tile_ok(h->p.lattice, compacted3d(h->p), tile_y, chunk_z))
        return h->fail(LBM_MS_E_ARG, "launch shape (%d, %d) not compiled for this lattice and storage",
                       tile_y, chunk_z);
    h->ty = tile_y;
    h->cz = chunk_z;
    int rc = h->upload_tiles();
    if (rc) return rc;
    return h->upload_tables();
}

int lbm_ms_set_geometry(lbm_ms_t h, const uint8_t* solid_host)
{
    if (!h || !solid_host) return LBM_MS_E_ARG;
    h->mask.assign(solid_host, solid_host + h->N);
    for (auto& v : h->mask) v = v ? 1 : 0;
    if (h->p.inlet_mode == LBM_MS_INLET_DIRICHLET) {
        h->n_open = clean_pores(h->p, h->mask);
        if (h->n_open <= 0) {
            h->geom = false;
            return h->fail(LBM_MS_E_GEOM, "no fluid path from the inlet column to the outlet column");
        }
    } else {
        h->n_open = 0;
        for (long long n = h->p.nx - 1; n < h->N; n += h->p.nx) h->n_open += h->mask[n] ? 0 : 1;
    }
    std::vector<int32_t> idx;
    h->n_fluid = build_index(h->mask, h->p.nx, h->p.ny, h->p.nz, idx);
    h->P = plane_pitch(h->n_fluid);
    h->S[0] = h->S[1] = 0.0;  // a source layer belongs to the geometry it was set on
    h->src_x0 = 1 << 30;
    h->n_src = 0;
    // the kernels address a population buffer and the NODE-shift references with 32-bit byte
    // offsets from their bases
    const unsigned long long fbytes = 2ull * h->q * (unsigned long long)h->P * elem_bytes(h->p.precision);
    const unsigned long long xbytes = node_shift(h->p) ? 16ull * (unsigned long long)h->n_fluid : 0ull;
    if (fbytes > (1ull << 32) || xbytes > (1ull << 32)) {
        h->geom = false;
        return h->fail(LBM_MS_E_ARG,
                       "%lld fluid nodes: one population buffer would take %llu bytes, beyond the "
                       "4 GiB that 32-bit offsets address", h->n_fluid, fbytes);
    }
    int rc = h->hip(hipMemcpyAsync(h->at(h->L.idx), idx.data(), idx.size() * sizeof(int32_t),
                                   hipMemcpyHostToDevice, h->stream), "index upload");
    if (rc) return rc;
    std::vector<int32_t> vox;
    if (h->p.advection) {  // the voxel of each compact node, for the advective passes
        vox.assign((size_t)h->n_fluid, 0);
        for (size_t n = 0; n < idx.size(); ++n)
            if (idx[n] >= 0) vox[(size_t)idx[n]] = (int32_t)n;
        if (!vox.empty()) {
            rc = h->hip(hipMemcpyAsync(h->at(h->L.vox), vox.data(), vox.size() * sizeof(int32_t),
                                       hipMemcpyHostToDevice, h->stream), "voxel list upload");
            if (rc) return rc;
        }
    }
    rc = h->sync();
    if (rc) return rc;
    h->geom = true;
    h->ready = false;
    rc = h->upload_tiles();
    if (rc) return rc;
    return h->upload_tables();
}

int lbm_ms_clean_geometry(int lattice, int nx, int ny, int nz, const uint8_t* solid_in,
                          uint8_t* solid_out, int64_t* n_open)
{
    if (!solid_in || !solid_out || nx < 2 || ny < 1 || nz < 1) return LBM_MS_E_ARG;
    if (!known_lattice(lattice)) return LBM_MS_E_ARG;
    if (is_2d(lattice) && nz != 1) return LBM_MS_E_ARG;
    lbm_ms_params p{};
    p.lattice = lattice;
    p.nx = nx;
    p.ny = ny;
    p.nz = nz;
    const size_t N = (size_t)nx * ny * nz;
    std::vector<uint8_t> m(solid_in, solid_in + N);
    for (auto& v : m) v = v ? 1 : 0;
    const long long open = clean_pores(p, m);
    std::memcpy(solid_out, m.data(), N);
    if (n_open) *n_open = open;
    return LBM_MS_OK;
}

int lbm_ms_work_list(int lattice, int nx, int ny, const uint8_t* solid, int tile_y, int rows,
                     int64_t* n_tiles, int64_t* n_ent, int32_t* tiles, uint32_t* ent)
{
    if (!solid || !n_tiles || !n_ent || nx < 2 || ny < 1) return LBM_MS_E_ARG;
    if (!known_lattice(lattice) || !is_2d(lattice) || !tile_ok(lattice, false, tile_y, rows)) return LBM_MS_E_ARG;
    std::vector<uint8_t> m(solid, solid + (size_t)nx * ny);
    for (auto& v : m) v = v ? 1 : 0;
    std::vector<int4> tl;
    std::vector<uint32_t> en;
    build_tiles_2d(nx, ny, tile_y, rows, m, 0, 0, tl, en);
    if (!tiles_in_bounds(tl, en, tile_y, rows)) return LBM_MS_E_ARG;
    *n_tiles = (int64_t)(tl.size() / 2);
    *n_ent = (int64_t)en.size();
    if (tiles)
        for (size_t t = 0; t < tl.size(); ++t) {
            tiles[4 * t + 0] = tl[t].x;
            tiles[4 * t + 1] = tl[t].y;
            tiles[4 * t + 2] = tl[t].z;
            tiles[4 * t + 3] = tl[t].w;
        }
    if (ent) std::memcpy(ent, en.data(), en.size() * sizeof(uint32_t));
    return LBM_MS_OK;
}

int lbm_ms_get_geometry(lbm_ms_t h, uint8_t* solid_host)
{
    if (!h || !solid_host) return LBM_MS_E_ARG;
    if (!h->geom) return h->fail(LBM_MS_E_STATE, "set_geometry first");
    std::memcpy(solid_host, h->mask.data(), h->N);
    return LBM_MS_OK;
}

int lbm_ms_set_bc(lbm_ms_t h, const double X_in[3], double j)
{
    if (!h || !X_in) return LBM_MS_E_ARG;
    if (!h->geom) return h->fail(LBM_MS_E_STATE, "set_geometry first");
    for (int s = 0; s < 3; ++s)
        if (!(X_in[s] >= 0.0)) return h->fail(LBM_MS_E_ARG, "X_in must be >= 0");
    if (std::fabs(X_in[0] + X_in[1] + X_in[2] - 1.0) > 1e-12)
        return h->fail(LBM_MS_E_ARG, "X_in must sum to 1");
    if (!(j >= 0.0) || !std::isfinite(j)) return h->fail(LBM_MS_E_ARG, "j must be finite and >= 0");
    for (int s = 0; s < 3; ++s) h->Xin[s] = X_in[s];
    h->j = j;
    // Eq. 39: N_s = -nu_s j / (n F); lattice flux per open outlet node
    const double face = (double)h->p.ny * h->p.nz;
    const double scale = h->n_open > 0 ? face / (double)h->n_open : 0.0;
    for (int s = 0; s < 2; ++s) {
        const double Ns = -(double)h->p.nu[s] * j / (h->p.n_electrons * FARADAY);
        h->Qs[s] = Ns * h->dt / (h->Ct * h->p.dx);
        h->Q[s] = h->Qs[s] * scale;
    }
    h->eps = h->p.eps_flux >= 0 ? h->p.eps_flux
                                : 1e-2 * std::max(std::fabs(h->Q[0]), std::fabs(h->Q[1])) + 1e-14;
    h->bc = true;
    return h->upload_tables();
}

int lbm_ms_set_source(lbm_ms_t h, int x_first, double j)
{
    if (!h) return LBM_MS_E_ARG;
    if (!h->geom) return h->fail(LBM_MS_E_STATE, "set_geometry first");
    if (h->p.advection) return h->fail(LBM_MS_E_ARG, "no volumetric source with advection");
    if (x_first < 0 || x_first > h->p.nx) return h->fail(LBM_MS_E_ARG, "x_first must lie in [0, nx]");
    if (!(j >= 0.0) || !std::isfinite(j)) return h->fail(LBM_MS_E_ARG, "j must be finite and >= 0");
    long long n = 0;
    for (long long k = 0; k < h->N; ++k)
        if (!h->mask[k] && (int)(k % h->p.nx) >= x_first) ++n;
    if (x_first < h->p.nx && n == 0) return h->fail(LBM_MS_E_ARG, "no fluid node in the source layer");
    h->n_src = x_first < h->p.nx ? n : 0;
    h->src_x0 = x_first < h->p.nx ? x_first : (1 << 30);
    // the layer's total per step is the electrode flux of Eq. 39 over the whole face:
    // S_s = -N_s dt n_face / (C_t dx n_layer), N_s = -nu_s j / (n F)
    const double face = (double)h->p.ny * h->p.nz;
    for (int s = 0; s < 2; ++s) {
        const double Ns = -(double)h->p.nu[s] * j / (h->p.n_electrons * FARADAY);
        h->S[s] = h->n_src > 0 ? -Ns * h->dt * face / (h->Ct * h->p.dx * (double)h->n_src) : 0.0;
    }
    return h->upload_tables();
}

static int init_common(lbm_ms_t h, const double* Xdev)
{
    h->cur = 0;
    StepArgs a = h->args(1);  // writes buffer 0 (fout of in_buf = 1)
    int rc = h->hip(launch_init(h->stream, a, h->p.lattice, h->prec(), h->ns(), Xdev, h->Xin[0],
                                h->Xin[1]), "init kernel");
    if (rc) return rc;
    if (h->p.advection) {  // velocity model at rest, zero velocities of both parities
        rc = h->hip(launch_adv_rest(h->stream, a, h->adv_args(1),
                                    reinterpret_cast<double*>(h->at(h->L.u[1])), h->p.lattice,
                                    h->prec()), "velocity model init");
        if (rc) return rc;
    }
    rc = h->hip(hipMemsetAsync(h->at(h->L.flags), 0, 64, h->stream), "flag reset");
    if (rc) return rc;
    // residual snapshot of the initial state
    StepArgs r = h->args(0);
    rc = h->hip(launch_residual(h->stream, r, h->p.lattice, h->prec(), h->ns(),
                                (double*)h->at(h->L.snap), 1, (double*)h->at(h->L.part),
                                RED_BLOCKS, (double*)h->at(h->L.scal)), "snapshot");
    if (rc) return rc;
    rc = h->sync();
    if (rc) return rc;
    h->steps = 0;
    h->snap_step = 0;
    h->ready = true;
    return LBM_MS_OK;
}

int lbm_ms_init(lbm_ms_t h, const double* X0, int on_device)
{
    if (!h) return LBM_MS_E_ARG;
    if (!h->geom || !h->bc) return h->fail(LBM_MS_E_STATE, "set_geometry and set_bc first");
    const double* Xdev = nullptr;
    if (X0) {
        if (on_device) {
            Xdev = X0;
        } else {
            int rc = h->hip(hipMemcpyAsync(h->at(h->L.field), X0, 3ull * h->N * sizeof(double),
                                           hipMemcpyHostToDevice, h->stream), "field upload");
            if (rc) return rc;
            Xdev = (const double*)h->at(h->L.field);
        }
    }
    return init_common(h, Xdev);
}

int lbm_ms_init_paper_profile(lbm_ms_t h)
{
    if (!h) return LBM_MS_E_ARG;
    if (!h->geom || !h->bc) return h->fail(LBM_MS_E_STATE, "set_geometry and set_bc first");
    StepArgs a = h->args(0);
    int rc = h->hip(launch_paper_profile(h->stream, a, h->Qs[0], h->Qs[1], (double*)h->at(h->L.prof),
                                         (double*)h->at(h->L.field)), "paper profile");
    if (rc) return rc;
    return init_common(h, (const double*)h->at(h->L.field));
}

int lbm_ms_paper_profile(lbm_ms_t h, double* prof)
{
    if (!h || !prof) return LBM_MS_E_ARG;
    if (!h->geom || !h->bc) return h->fail(LBM_MS_E_STATE, "set_geometry and set_bc first");
    StepArgs a = h->args(h->cur);
    // the profile kernel writes prof[2][nx]; the broadcast into the field buffer is harmless
    int rc = h->hip(launch_paper_profile(h->stream, a, h->Qs[0], h->Qs[1], (double*)h->at(h->L.prof),
                                         (double*)h->at(h->L.field)), "paper profile");
    if (rc) return rc;
    rc = h->hip(hipMemcpyAsync(prof, h->at(h->L.prof), 2ull * h->p.nx * sizeof(double),
                               hipMemcpyDeviceToHost, h->stream), "profile readback");
    if (rc) return rc;
    return h->sync();
}

int lbm_ms_step(lbm_ms_t h, int64_t nsteps)
{
    if (!h) return LBM_MS_E_ARG;
    if (!h->ready) return h->fail(LBM_MS_E_STATE, "init first");
    if (nsteps < 0) return h->fail(LBM_MS_E_ARG, "nsteps < 0");
    const int nb = h->nblocks_step();
    const StepArgs* tab = reinterpret_cast<const StepArgs*>(h->ws + h->L.inst);
    const int4* tiles = reinterpret_cast<const int4*>(h->ws + h->L.tiles);
    const unsigned* ent = reinterpret_cast<const unsigned*>(h->ws + h->L.ent);
    for (int64_t t = 0; t < nsteps; ++t) {
        hipError_t e;
        if (h->p.advection) {
            e = launch_adv_step(h->stream, h->args(h->cur), h->adv_args(h->cur),
                                reinterpret_cast<double*>(h->at(h->L.xa)), h->p.lattice, h->prec());
        } else if (is_2d(h->p.lattice)) {
            e = launch_step2d(h->stream, tab + h->cur, tiles, ent, h->ntiles, h->p.lattice, h->prec(),
                              h->ns(), h->ty, h->cz);
        } else {
            StepArgs a = h->args(h->cur);
            const bool cols = compacted_ty(h->ty);
            if (cols && h->c3_ty != h->ty) return h->fail(LBM_MS_E_STATE, "column lists not built");
            e = launch_step(h->stream, a, h->p.lattice, h->prec(), h->ns(), h->ty, h->cz, nb,
                            cols ? reinterpret_cast<const unsigned*>(h->ws + h->L.c3off) : nullptr,
                            cols ? reinterpret_cast<const unsigned short*>(h->ws + h->L.c3pos) : nullptr);
        }
        if (e != hipSuccess) return h->hip(e, "step kernel");
        h->cur ^= 1;
        ++h->steps;
    }
    return LBM_MS_OK;
}

int lbm_ms_time_steps(lbm_ms_t h, int64_t nsteps, double* ms)
{
    if (!h || !ms) return LBM_MS_E_ARG;
    hipEvent_t e0, e1;
    int rc = h->hip(hipEventCreate(&e0), "event");
    if (rc) return rc;
    rc = h->hip(hipEventCreate(&e1), "event");
    if (rc) { hipEventDestroy(e0); return rc; }
    hipEventRecord(e0, h->stream);
    rc = lbm_ms_step(h, nsteps);
    hipEventRecord(e1, h->stream);
    if (!rc) rc = h->hip(hipEventSynchronize(e1), "event sync");
    float t = 0.f;
    if (!rc) rc = h->hip(hipEventElapsedTime(&t, e0, e1), "elapsed");
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    *ms = t;
    return rc;
}

// runs the residual reduction; vals[0..5] as in k_residual
// queues the residual reduction and the read-backs of its sums and of the clamp flag into the
// pinned buffer (read once the stream has been synchronized)
static int reduce_launch(lbm_ms_t h, int update)
{
    StepArgs a = h->args(h->cur);
    int rc = h->hip(launch_residual(h->stream, a, h->p.lattice, h->prec(), h->ns(),
                                    (double*)h->at(h->L.snap), update, (double*)h->at(h->L.part),
                                    RED_BLOCKS, (double*)h->at(h->L.scal)), "residual");
    if (rc) return rc;
    rc = h->hip(hipMemcpyAsync(h->pinned, h->at(h->L.scal), 8 * sizeof(double),
                               hipMemcpyDeviceToHost, h->stream), "residual readback");
    if (rc) return rc;
    return h->hip(hipMemcpyAsync(h->pinned + 8, h->at(h->L.flags), 16, hipMemcpyDeviceToHost,
                                 h->stream), "flag readback");
}

static int reduce_state(lbm_ms_t h, int update, double* vals)
{
    int rc = reduce_launch(h, update);
    if (rc) return rc;
    rc = h->sync();
    if (rc) return rc;
    std::memcpy(vals, h->pinned, 6 * sizeof(double));
    return LBM_MS_OK;
}

// The check of a window whose reduction reduce_launch queued and the stream has completed: the
// residual from the pinned sums, then the status (the clamp flag is cleared for the next window).
static int residual_eval(lbm_ms_t h, double* residual)
{
    double v[6];
    std::memcpy(v, h->pinned, 6 * sizeof(double));
    int rc = LBM_MS_OK;
    const unsigned clamp = ((const unsigned*)(h->pinned + 8))[0];
    const long long K = h->steps - h->snap_step;
    h->snap_step = h->steps;
    const double r = (K > 0 && v[1] > 0) ? std::sqrt(v[0]) / ((double)K * std::sqrt(v[1])) : 0.0;
    *residual = r;
    // the clamp flag covers one check window: clear it whatever this check reports
    if (clamp) {
        rc = h->hip(hipMemsetAsync(h->at(h->L.flags), 0, 64, h->stream), "clamp flag reset");
        if (rc) return rc;
    }
    if (v[4] > 0 || !std::isfinite(r))
        return h->fail(LBM_MS_E_DIVERGED, "%.0f nodes with non-finite mole fractions", v[4]);
    if (v[5] > 0)
        return h->fail(LBM_MS_E_NEG_FRACTION, "%.0f nodes with a mole fraction below -1e-12", v[5]);
    if (clamp) return h->fail(LBM_MS_E_TAU_CLAMP, "a relaxation time hit the clamp");
    return LBM_MS_OK;
}

int lbm_ms_residual(lbm_ms_t h, double* residual)
{
    if (!h || !residual) return LBM_MS_E_ARG;
    if (!h->ready) return h->fail(LBM_MS_E_STATE, "init first");
    int rc = reduce_launch(h, 1);
    if (rc) return rc;
    rc = h->sync();
    if (rc) return rc;
    return residual_eval(h, residual);
}

int lbm_ms_converge(lbm_ms_t h, double tol, int64_t max_steps, int check_every,
                    int64_t* steps_taken, double* residual)
{
    if (!h || check_every <= 0 || max_steps < 0) return LBM_MS_E_ARG;
    if (!h->ready) return h->fail(LBM_MS_E_STATE, "init first");
    // start a fresh window
    double v[6];
    int rc = reduce_state(h, 1, v);
    if (rc) return rc;
    h->snap_step = h->steps;
    int64_t taken = 0;
    double r = INFINITY;
    while (taken < max_steps) {
        const int64_t n = std::min<int64_t>(check_every, max_steps - taken);
        rc = lbm_ms_step(h, n);
        if (rc) break;
        taken += n;
        rc = lbm_ms_residual(h, &r);
        if (rc) break;
        if (r < tol) break;
    }
    if (steps_taken) *steps_taken = taken;
    if (residual) *residual = r;
    if (rc) return rc;
    if (!(r < tol)) return h->fail(LBM_MS_E_NOT_CONVERGED, "residual %.3e after %lld steps", r, (long long)taken);
    return LBM_MS_OK;
}

static int faces(lbm_ms_t h, double* v)
{
    StepArgs a = h->args(h->cur);
    int rc = h->hip(launch_faces(h->stream, a, h->p.lattice, h->prec(), h->ns(), (double*)h->at(h->L.part),
                                 RED_BLOCKS, (double*)h->at(h->L.scal) + 8), "face reduction");
    if (rc) return rc;
    rc = h->hip(hipMemcpyAsync(h->pinned, (double*)h->at(h->L.scal) + 8, 8 * sizeof(double),
                               hipMemcpyDeviceToHost, h->stream), "face readback");
    if (rc) return rc;
    rc = h->sync();
    if (rc) return rc;
    std::memcpy(v, h->pinned, 7 * sizeof(double));
    return LBM_MS_OK;
}

int lbm_ms_outlet_mean(lbm_ms_t h, double X_out[3])
{
    if (!h || !X_out) return LBM_MS_E_ARG;
    if (!h->ready) return h->fail(LBM_MS_E_STATE, "init first");
    double v[7];
    int rc = faces(h, v);
    if (rc) return rc;
    if (v[2] <= 0) return h->fail(LBM_MS_E_GEOM, "no open outlet node");
    X_out[0] = v[0] / v[2];
    X_out[1] = v[1] / v[2];
    X_out[2] = 1.0 - X_out[0] - X_out[1];
    return LBM_MS_OK;
}

int lbm_ms_overpotential(lbm_ms_t h, double* eta)
{
    if (!h || !eta) return LBM_MS_E_ARG;
    double Xo[3];
    int rc = lbm_ms_outlet_mean(h, Xo);
    if (rc) return rc;
    if (!(Xo[0] > 0 && Xo[1] > 0 && h->Xin[0] > 0 && h->Xin[1] > 0))
        return h->fail(LBM_MS_E_NEG_FRACTION, "non-positive mole fraction in Eq. 43");
    // Eq. 43
    *eta = (R_GAS * h->p.T / (h->p.n_electrons * FARADAY)) *
           std::log(h->Xin[0] * Xo[1] / (Xo[0] * h->Xin[1]));
    return LBM_MS_OK;
}

int lbm_ms_mass_balance(lbm_ms_t h, double inventory[2], double inflow[2], double outflow[2])
{
    if (!h) return LBM_MS_E_ARG;
    if (!h->ready) return h->fail(LBM_MS_E_STATE, "init first");
    double v[6], f[7];
    int rc = reduce_state(h, 0, v);
    if (rc) return rc;
    rc = faces(h, f);
    if (rc) return rc;
    // the stored state is post-collision: the layer's nodes hold this step's source already
    if (inventory) { inventory[0] = v[2] - (double)h->n_src * h->S[0]; inventory[1] = v[3] - (double)h->n_src * h->S[1]; }
    if (inflow) { inflow[0] = f[3]; inflow[1] = f[4]; }
    if (outflow) { outflow[0] = f[5]; outflow[1] = f[6]; }
    return LBM_MS_OK;
}

int lbm_ms_get_fields(lbm_ms_t h, double* X, int on_device)
{
    if (!h || !X) return LBM_MS_E_ARG;
    if (!h->ready) return h->fail(LBM_MS_E_STATE, "init first");
    StepArgs a = h->args(h->cur);
    double* dst = on_device ? X : (double*)h->at(h->L.field);
    int rc = h->hip(launch_fields(h->stream, a, h->p.lattice, h->prec(), h->ns(), dst), "fields");
    if (rc) return rc;
    if (!on_device) {
        rc = h->hip(hipMemcpyAsync(X, dst, 3ull * h->N * sizeof(double), hipMemcpyDeviceToHost, h->stream),
                    "field readback");
        if (rc) return rc;
    }
    return h->sync();
}

int lbm_ms_get_velocity(lbm_ms_t h, double* u)
{
    if (!h || !u) return LBM_MS_E_ARG;
    if (!h->p.advection) return h->fail(LBM_MS_E_STATE, "no velocity model without advection");
    if (!h->ready) return h->fail(LBM_MS_E_STATE, "init first");
    // after a step of parity c the buffer u[1 - c] holds this step's node velocity, u[c] the
    // previous one; with h->cur already flipped, u[cur] is the latest
    StepArgs a = h->args(h->cur);
    double* dst = (double*)h->at(h->L.field);
    const double scale = h->p.dx / h->dt;  // lattice velocity to m/s
    int rc = h->hip(launch_adv_velocity(h->stream, a, (const double*)h->at(h->L.u[h->cur]),
                                        (const double*)h->at(h->L.u[1 - h->cur]), scale, dst,
                                        h->p.lattice, h->prec()), "velocity");
    if (rc) return rc;
    rc = h->hip(hipMemcpyAsync(u, dst, 3ull * h->N * sizeof(double), hipMemcpyDeviceToHost, h->stream),
                "velocity readback");
    if (rc) return rc;
    return h->sync();
}

int lbm_ms_get_populations(lbm_ms_t h, double* f)
{
    if (!h || !f) return LBM_MS_E_ARG;
    if (!h->ready) return h->fail(LBM_MS_E_STATE, "init first");
    StepArgs a = h->args(h->cur);
    double* tmp = (double*)h->at(h->L.field);
    for (int s = 0; s < 2; ++s)
        for (int k = 0; k < h->q; ++k) {
            int rc = h->hip(launch_populations(h->stream, a, h->p.lattice, h->prec(), h->ns(), s, k, tmp),
                            "populations");
            if (rc) return rc;
            rc = h->hip(hipMemcpyAsync(f + ((size_t)s * h->q + k) * h->N, tmp, h->N * sizeof(double),
                                       hipMemcpyDeviceToHost, h->stream), "population readback");
            if (rc) return rc;
            rc = h->sync();
            if (rc) return rc;
        }
    return LBM_MS_OK;
}

// checkpoint blob: header | populations | node shift field | residual snapshot
struct StateHeader {
    uint64_t magic, hash;
    int64_t steps, snap_step;
    uint64_t fbytes, xbytes, sbytes;
};

int lbm_ms_save_state(lbm_ms_t h, void* buf, size_t* bytes)
{
    if (!h || !bytes) return LBM_MS_E_ARG;
    if (h->p.advection) return h->fail(LBM_MS_E_STATE, "no checkpoints with advection");
    const size_t fb = 2ull * h->q * h->P * elem_bytes(h->p.precision);
    const size_t xb = node_shift(h->p) ? 2ull * h->n_fluid * sizeof(double) : 0;
    const size_t sb = 2ull * h->n_fluid * sizeof(double);
    const size_t need = sizeof(StateHeader) + fb + xb + sb;
    if (!buf) { *bytes = need; return LBM_MS_OK; }
    if (*bytes < need) return h->fail(LBM_MS_E_ARG, "buffer too small (%zu < %zu)", *bytes, need);
    if (!h->ready) return h->fail(LBM_MS_E_STATE, "init first");
    StateHeader H{STATE_MAGIC, param_hash(h->p, h->n_fluid), h->steps, h->snap_step, fb, xb, sb};
    char* c = (char*)buf;
    std::memcpy(c, &H, sizeof(H));
    c += sizeof(H);
    int rc = h->hip(hipMemcpyAsync(c, h->at(h->L.f[h->cur]), fb, hipMemcpyDeviceToHost, h->stream), "save");
    if (rc) return rc;
    c += fb;
    if (xb) {
        rc = h->hip(hipMemcpyAsync(c, h->at(h->L.xn[h->cur]), xb, hipMemcpyDeviceToHost, h->stream), "save");
        if (rc) return rc;
        c += xb;
    }
    rc = h->hip(hipMemcpyAsync(c, h->at(h->L.snap), sb, hipMemcpyDeviceToHost, h->stream), "save");
    if (rc) return rc;
    *bytes = need;
    return h->sync();
}

int lbm_ms_load_state(lbm_ms_t h, const void* buf, size_t bytes)
{
    if (!h || !buf) return LBM_MS_E_ARG;
    if (h->p.advection) return h->fail(LBM_MS_E_STATE, "no checkpoints with advection");
    if (!h->geom || !h->bc) return h->fail(LBM_MS_E_STATE, "set_geometry and set_bc first");
    StateHeader H;
    if (bytes < sizeof(H)) return h->fail(LBM_MS_E_ARG, "blob too small");
    std::memcpy(&H, buf, sizeof(H));
    const size_t fb = 2ull * h->q * h->P * elem_bytes(h->p.precision);
    const size_t xb = node_shift(h->p) ? 2ull * h->n_fluid * sizeof(double) : 0;
    const size_t sb = 2ull * h->n_fluid * sizeof(double);
    if (H.magic != STATE_MAGIC || H.hash != param_hash(h->p, h->n_fluid) || H.fbytes != fb || H.xbytes != xb ||
        H.sbytes != sb || bytes < sizeof(H) + fb + xb + sb)
        return h->fail(LBM_MS_E_ARG, "checkpoint does not match this handle");
    const char* c = (const char*)buf + sizeof(H);
    h->cur = 0;
    int rc = h->hip(hipMemcpyAsync(h->at(h->L.f[0]), c, fb, hipMemcpyHostToDevice, h->stream), "load");
    if (rc) return rc;
    c += fb;
    if (xb) {
        rc = h->hip(hipMemcpyAsync(h->at(h->L.xn[0]), c, xb, hipMemcpyHostToDevice, h->stream), "load");
        if (rc) return rc;
        c += xb;
    }
    rc = h->hip(hipMemcpyAsync(h->at(h->L.snap), c, sb, hipMemcpyHostToDevice, h->stream), "load");
    if (rc) return rc;
    rc = h->hip(hipMemsetAsync(h->at(h->L.flags), 0, 64, h->stream), "flag reset");
    if (rc) return rc;
    rc = h->sync();
    if (rc) return rc;
    h->steps = H.steps;
    h->snap_step = H.snap_step;
    h->ready = true;
    return LBM_MS_OK;
}

int lbm_ms_get_info(lbm_ms_t h, lbm_ms_info* info)
{
    if (!h || !info) return LBM_MS_E_ARG;
    std::memset(info, 0, sizeof(*info));
    info->dt = h->dt;
    info->Ct = h->Ct;
    for (int i = 0; i < 9; ++i) info->Dl[i] = h->Dl[i];
    info->Q[0] = h->Q[0];
    info->Q[1] = h->Q[1];
    info->eps_flux = h->eps;
    info->n_fluid = h->n_fluid;
    info->n_open_outlet = h->n_open;
    info->steps = h->steps;
    info->q = h->q;
    info->tile_x = 64;
    info->tile_y = h->ty;
    info->chunk_z = h->cz;
    info->workspace_bytes = h->L.total;
    info->S[0] = h->S[0];
    info->S[1] = h->S[1];
    info->n_source = h->n_src;
    info->source_x0 = h->src_x0 < h->p.nx ? h->src_x0 : h->p.nx;
    return LBM_MS_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------------------------
// batched solves
// ---------------------------------------------------------------------------------------------
struct lbm_ms_batch_s {
    lbm_ms_params common{};
    hipStream_t user = nullptr;  // caller's stream
    hipStream_t stream = nullptr;  // the batch's own stream (graph capture needs a non-legacy one)
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    std::vector<lbm_ms_s*> inst;
    std::vector<std::vector<int4>> tiles_k;
    char* ws = nullptr;
    size_t off_tab = 0, off_tiles = 0, off_ent = 0;
    size_t off_slots = 0, off_res = 0;  // batched residual check: slot table, results [count][16]
    double* pinned = nullptr;           // host copy of the results
    size_t tile_cap = 0, ent_cap = 0;
    int count = 0, ty = 0, rows = 0;  // rows > 0: packed tiles of at most `rows` rows
    std::vector<char> active;
    std::vector<int> retired_status;  // why an inactive instance left the work list
    int ntiles = 0;
    int cur = 0;
    bool use_graphs = true;
    hipGraphExec_t gexec[2] = {nullptr, nullptr};
    int graph_len = 0;
    std::string err;

    int fail(int code, const std::string& m) { err = m; return code; }
    int hip(hipError_t e, const char* what)
    {
        if (e == hipSuccess) return LBM_MS_OK;
        return fail(LBM_MS_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
    }
    // order the batch stream after the caller's stream
    int enter()
    {
        int rc = hip(hipEventRecord(ev_in, user), "event record");
        if (rc) return rc;
        return hip(hipStreamWaitEvent(stream, ev_in, 0), "stream wait");
    }
    // order the caller's stream after the batch stream
    int leave(int rc)
    {
        if (hipEventRecord(ev_out, stream) == hipSuccess) (void)hipStreamWaitEvent(user, ev_out, 0);
        return rc;
    }
    void drop_graphs()
    {
        for (auto& g : gexec)
            if (g) { (void)hipGraphExecDestroy(g); g = nullptr; }
        graph_len = 0;
    }
    int upload_tables()
    {
        std::vector<StepArgs> t(2 * (size_t)count);
        for (int k = 0; k < count; ++k) {
            t[k] = inst[k]->args(0);
            t[count + k] = inst[k]->args(1);
        }
        int rc = hip(hipStreamSynchronize(stream), "sync");
        if (rc) return rc;
        rc = hip(hipMemcpy(ws + off_tab, t.data(), t.size() * sizeof(StepArgs), hipMemcpyHostToDevice),
                 "instance table upload");
        return rc;
    }
    // work list of the active instances (host compaction of the per-instance tile lists)
    int upload_active_tiles()
    {
        std::vector<int4> tl;
        for (int k = 0; k < count; ++k)
            if (active[k]) tl.insert(tl.end(), tiles_k[k].begin(), tiles_k[k].end());
        if (tl.size() / 2 > tile_cap) return fail(LBM_MS_E_NOMEM, "tile list exceeds its share");
        int rc = hip(hipStreamSynchronize(stream), "sync");
        if (rc) return rc;
        if (!tl.empty()) {
            rc = hip(hipMemcpy(ws + off_tiles, tl.data(), tl.size() * sizeof(int4), hipMemcpyHostToDevice),
                     "tile upload");
            if (rc) return rc;
        }
        ntiles = (int)(tl.size() / 2);
        drop_graphs();
        return LBM_MS_OK;
    }
    int upload_lists()
    {
        std::vector<uint32_t> en;
        tiles_k.assign(count, {});
        for (int k = 0; k < count; ++k)
            build_tiles_2d(inst[k]->p.nx, inst[k]->p.ny, ty, rows, inst[k]->mask, k, 0, tiles_k[k], en);
        if (en.size() > ent_cap) return fail(LBM_MS_E_NOMEM, "entry list exceeds its share");
        for (int k = 0; k < count; ++k)
            if (!tiles_in_bounds(tiles_k[k], en, ty, rows))
                return fail(LBM_MS_E_ARG, "work list of instance " + std::to_string(k) + " out of bounds");
        int rc = hip(hipStreamSynchronize(stream), "sync");
        if (rc) return rc;
        rc = hip(hipMemcpy(ws + off_ent, en.data(), en.size() * sizeof(uint32_t), hipMemcpyHostToDevice),
                 "entry upload");
        if (rc) return rc;
        return upload_active_tiles();
    }
    // the residual slots of the instances (pointers into their workspaces, on / off the list)
    int upload_slots()
    {
        std::vector<ResidualSlot> t(count);
        for (int k = 0; k < count; ++k) {
            lbm_ms_s* h = inst[k];
            t[k].snap = reinterpret_cast<double*>(h->at(h->L.snap));
            t[k].partial = reinterpret_cast<double*>(h->at(h->L.part));
            t[k].flags = reinterpret_cast<const unsigned*>(h->at(h->L.flags));
            t[k].active = active[k] ? 1 : 0;
            t[k].pad = 0;
        }
        int rc = hip(hipStreamSynchronize(stream), "sync");
        if (rc) return rc;
        return hip(hipMemcpy(ws + off_slots, t.data(), t.size() * sizeof(ResidualSlot),
                             hipMemcpyHostToDevice), "slot upload");
    }
    // every active instance's residual window reduced in two launches and read back at once; on
    // return each active instance's pinned page holds what reduce_launch would have put there
    int check_all()
    {
        const StepArgs* tab = reinterpret_cast<const StepArgs*>(ws + off_tab) + (size_t)cur * count;
        int rc = hip(launch_residual_batch(stream, tab, reinterpret_cast<const ResidualSlot*>(ws + off_slots),
                                           count, common.lattice, common.precision,
                                           node_shift(common) ? 1 : 0, 1, RED_BLOCKS,
                                           reinterpret_cast<double*>(ws + off_res)), "batched residual");
        if (rc) return rc;
        rc = hip(hipMemcpyAsync(pinned, ws + off_res, (size_t)count * 16 * sizeof(double),
                                hipMemcpyDeviceToHost, stream), "residual readback");
        if (rc) return rc;
        rc = hip(hipStreamSynchronize(stream), "residual sync");
        if (rc) return rc;
        for (int k = 0; k < count; ++k)
            if (active[k]) std::memcpy(inst[k]->pinned, pinned + (size_t)k * 16, 10 * sizeof(double));
        return LBM_MS_OK;
    }
    hipError_t launch_one()
    {
        const StepArgs* tab = reinterpret_cast<const StepArgs*>(ws + off_tab) + (size_t)cur * count;
        return launch_step2d(stream, tab, reinterpret_cast<const int4*>(ws + off_tiles),
                             reinterpret_cast<const unsigned*>(ws + off_ent), ntiles, common.lattice,
                             common.precision, node_shift(common) ? 1 : 0, ty, rows);
    }
    void advance(int64_t n)
    {
        if (n & 1) cur ^= 1;
        for (int k = 0; k < count; ++k)
            if (active[k]) {
                inst[k]->cur = cur;
                inst[k]->steps += n;
            }
    }
    int step_eager(int64_t n)
    {
        for (int64_t t = 0; t < n; ++t) {
            const hipError_t e = launch_one();
            if (e != hipSuccess) return hip(e, "batched step");
            cur ^= 1;
        }
        if (n & 1) cur ^= 1;  // advance() applies the parity change once
        advance(n);
        return LBM_MS_OK;
    }
    // n steps as one hipGraph (captured once per start parity, active set and length)
    int step_graph(int n)
    {
        if (graph_len != n) drop_graphs();
        const int p0 = cur;
        if (!gexec[p0]) {
            hipGraph_t g = nullptr;
            int rc = hip(hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal), "begin capture");
            if (rc) return rc;
            hipError_t le = hipSuccess;
            for (int t = 0; t < n && le == hipSuccess; ++t) {
                le = launch_one();
                cur ^= 1;
            }
            cur = p0;
            const hipError_t ce = hipStreamEndCapture(stream, &g);
            if (le != hipSuccess) { if (g) (void)hipGraphDestroy(g); return hip(le, "captured launch"); }
            rc = hip(ce, "end capture");
            if (rc) return rc;
            rc = hip(hipGraphInstantiate(&gexec[p0], g, nullptr, nullptr, 0), "graph instantiate");
            (void)hipGraphDestroy(g);
            if (rc) return rc;
            graph_len = n;
        }
        int rc = hip(hipGraphLaunch(gexec[p0], stream), "graph launch");
        if (rc) return rc;
        advance(n);
        return LBM_MS_OK;
    }
};

namespace {

size_t instance_bytes(const lbm_ms_params& common, const lbm_ms_instance_desc& d, lbm_ms_params* out)
{
    lbm_ms_params p = common;
    p.nx = d.nx;
    p.ny = d.ny;
    p.nz = 1;
    if (out) *out = p;
    return lbm_ms_workspace_bytes(&p);
}

bool batch_layout(const lbm_ms_params* common, const lbm_ms_instance_desc* inst, int count,
                  std::vector<size_t>* offs, size_t* off_tab, size_t* off_tiles, size_t* off_ent,
                  size_t* off_slots, size_t* off_res, size_t* tile_cap, size_t* ent_cap, size_t* total)
{
    // batches step through the tile work list, which has no advective coupling
    if (!common || !inst || count <= 0 || !is_2d(common->lattice) || common->advection) return false;
    size_t off = 0, tc = 0, ec = 0;
    auto take = [&](size_t b) { size_t o = off; off += (b + 255) & ~(size_t)255; return o; };
    if (offs) offs->clear();
    for (int k = 0; k < count; ++k) {
        const size_t b = instance_bytes(*common, inst[k], nullptr);
        if (b == 0 || !inst[k].solid) return false;
        const size_t o = take(b);
        if (offs) offs->push_back(o);
        size_t t = 0, e = 0;
        tile_caps(inst[k].nx, inst[k].ny, &t, &e);
        tc += t;
        ec += e;
    }
    const size_t ot = take(2ull * count * sizeof(StepArgs));
    const size_t oti = take(tc * 2 * sizeof(int4));
    const size_t oe = take(ec * sizeof(uint32_t));
    const size_t osl = take((size_t)count * sizeof(ResidualSlot));
    const size_t ore = take((size_t)count * 16 * sizeof(double));
    if (off_slots) *off_slots = osl;
    if (off_res) *off_res = ore;
    if (off_tab) *off_tab = ot;
    if (off_tiles) *off_tiles = oti;
    if (off_ent) *off_ent = oe;
    if (tile_cap) *tile_cap = tc;
    if (ent_cap) *ent_cap = ec;
    if (total) *total = off;
    return true;
}

}  // namespace

extern "C" {

size_t lbm_ms_batch_workspace_bytes(const lbm_ms_params* common, const lbm_ms_instance_desc* inst,
                                    int count)
{
    size_t total = 0;
    if (!batch_layout(common, inst, count, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
                      nullptr, &total)) {
        g_create_err = "invalid batch parameters (D2Q9 common parameters, count > 0, every instance "
                       "valid with a solid mask)";
        return 0;
    }
    return total;
}

void lbm_ms_batch_destroy(lbm_ms_batch_t b)
{
    if (!b) return;
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    b->drop_graphs();
    for (auto* h : b->inst) lbm_ms_destroy(h);
    if (b->ev_in) (void)hipEventDestroy(b->ev_in);
    if (b->ev_out) (void)hipEventDestroy(b->ev_out);
    if (b->stream) (void)hipStreamDestroy(b->stream);
    if (b->pinned) (void)hipHostFree(b->pinned);
    delete b;
}

int lbm_ms_batch_create(const lbm_ms_params* common, const lbm_ms_instance_desc* inst, int count,
                        void* d_workspace, size_t bytes, lbm_ms_batch_t* out)
{
    g_create_err.clear();
    if (!out) return create_fail(LBM_MS_E_ARG, "out is NULL");
    *out = nullptr;
    std::vector<size_t> offs;
    size_t ot, oti, oe, osl, ore, tc, ec, total;
    if (!batch_layout(common, inst, count, &offs, &ot, &oti, &oe, &osl, &ore, &tc, &ec, &total))
        return create_fail(LBM_MS_E_ARG, "invalid batch parameters (2D common parameters without "
                                         "advection, count > 0, every instance valid with a solid "
                                         "mask)");
    if (!d_workspace || ((uintptr_t)d_workspace & 255))
        return create_fail(LBM_MS_E_ARG, "workspace is NULL or not 256-byte aligned");
    if (bytes < total)
        return create_fail(LBM_MS_E_NOMEM, "workspace of " + std::to_string(bytes) + " bytes, " +
                                               std::to_string(total) + " needed");
    lbm_ms_batch_s* b = new (std::nothrow) lbm_ms_batch_s();
    if (!b) return create_fail(LBM_MS_E_NOMEM, "host allocation failed");
    b->common = *common;
    b->user = (hipStream_t)common->stream;
    b->ws = (char*)d_workspace;
    b->off_tab = ot;
    b->off_tiles = oti;
    b->off_ent = oe;
    b->off_slots = osl;
    b->off_res = ore;
    b->tile_cap = tc;
    b->ent_cap = ec;
    b->count = count;
    b->ty = default_tile_y(*common);
    b->rows = default_chunk_z(*common);
    if (b->ty > 16 || !tile_ok(common->lattice, false, b->ty, b->rows)) {
        b->ty = 8;
        b->rows = 0;
    }
    int rc = LBM_MS_OK;
    if (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&b->ev_out, hipEventDisableTiming) != hipSuccess) {
        lbm_ms_batch_destroy(b);
        return create_fail(LBM_MS_E_HIP, "stream or event creation failed");
    }
    if (hipHostMalloc((void**)&b->pinned, (size_t)count * 16 * sizeof(double)) != hipSuccess) {
        b->pinned = nullptr;
        lbm_ms_batch_destroy(b);
        return create_fail(LBM_MS_E_HIP, "hipHostMalloc of the residual readback failed");
    }
    rc = b->enter();
    for (int k = 0; k < count && rc == LBM_MS_OK; ++k) {
        lbm_ms_params pk;
        const size_t bk = instance_bytes(*common, inst[k], &pk);
        pk.stream = b->stream;
        pk.tile_y = b->ty;
        pk.chunk_z = b->rows;
        lbm_ms_t h = nullptr;
        rc = lbm_ms_create(&pk, b->ws + offs[k], bk, &h);
        if (rc) { b->err = "instance " + std::to_string(k) + ": create failed"; break; }
        b->inst.push_back(h);
        rc = lbm_ms_set_geometry(h, inst[k].solid);
        if (rc == LBM_MS_OK) rc = lbm_ms_set_bc(h, inst[k].X_in, inst[k].j_A_per_m2);
        if (rc) b->err = "instance " + std::to_string(k) + ": " + h->err;
    }
    if (rc == LBM_MS_OK) {
        b->active.assign(count, 1);
        b->retired_status.assign(count, LBM_MS_OK);
        rc = b->upload_lists();
    }
    if (rc == LBM_MS_OK) rc = b->upload_tables();
    if (rc == LBM_MS_OK) rc = b->upload_slots();
    if (rc) {
        const std::string e = b->err.empty() ? std::string(lbm_ms_status_string(rc)) : b->err;
        lbm_ms_batch_destroy(b);
        return create_fail(rc, e);
    }
    *out = b;
    return b->leave(LBM_MS_OK);
}

const char* lbm_ms_batch_last_error(lbm_ms_batch_t b)
{
    if (b) return b->err.c_str();
    return g_create_err.empty() ? "null batch" : g_create_err.c_str();
}

lbm_ms_t lbm_ms_batch_instance(lbm_ms_batch_t b, int k)
{
    if (!b || k < 0 || k >= b->count) return nullptr;
    return b->inst[k];
}

int lbm_ms_batch_stats(lbm_ms_batch_t b, int* active, int64_t* fluid, int* tiles)
{
    if (!b) return LBM_MS_E_ARG;
    int a = 0;
    int64_t nf = 0;
    for (int k = 0; k < b->count; ++k)
        if (b->active[k]) { ++a; nf += b->inst[k]->n_fluid; }
    if (active) *active = a;
    if (fluid) *fluid = nf;
    if (tiles) *tiles = b->ntiles;
    return LBM_MS_OK;
}

int lbm_ms_batch_set_tile(lbm_ms_batch_t b, int tile_y, int rows)
{
    if (!b) return LBM_MS_E_ARG;
    if (!tile_ok(b->common.lattice, false, tile_y, rows)) return b->fail(LBM_MS_E_ARG, "launch shape not compiled");
    int rc = b->enter();
    if (rc) return rc;
    b->ty = tile_y;
    b->rows = rows;
    for (auto* h : b->inst) {
        h->ty = tile_y;
        h->cz = rows;
    }
    rc = b->upload_lists();
    return b->leave(rc);
}

int lbm_ms_batch_use_graphs(lbm_ms_batch_t b, int enable)
{
    if (!b) return LBM_MS_E_ARG;
    b->use_graphs = enable != 0;
    return LBM_MS_OK;
}

int lbm_ms_batch_init(lbm_ms_batch_t b, const double* X0, int on_device)
{
    if (!b) return LBM_MS_E_ARG;
    int rc = b->enter();
    if (rc) return rc;
    size_t off = 0;
    for (int k = 0; k < b->count && rc == LBM_MS_OK; ++k) {
        lbm_ms_t h = b->inst[k];
        rc = lbm_ms_init(h, X0 ? X0 + off : nullptr, on_device);
        if (rc) b->err = "instance " + std::to_string(k) + ": " + h->err;
        off += 3ull * h->N;
    }
    if (rc == LBM_MS_OK) {
        b->cur = 0;
        b->active.assign(b->count, 1);
        b->retired_status.assign(b->count, LBM_MS_OK);
        rc = b->upload_active_tiles();
        if (rc == LBM_MS_OK) rc = b->upload_slots();
    }
    return b->leave(rc);
}

int lbm_ms_batch_step(lbm_ms_batch_t b, int64_t nsteps)
{
    if (!b || nsteps < 0) return LBM_MS_E_ARG;
    for (auto* h : b->inst)
        if (!h->ready) return b->fail(LBM_MS_E_STATE, "init first");
    int rc = b->enter();
    if (rc) return rc;
    rc = b->step_eager(nsteps);
    return b->leave(rc);
}

int lbm_ms_batch_time_steps(lbm_ms_batch_t b, int64_t nsteps, double* ms)
{
    if (!b || !ms || nsteps < 0) return LBM_MS_E_ARG;
    for (auto* h : b->inst)
        if (!h->ready) return b->fail(LBM_MS_E_STATE, "init first");
    hipEvent_t e0, e1;
    int rc = b->hip(hipEventCreate(&e0), "event");
    if (rc) return rc;
    rc = b->hip(hipEventCreate(&e1), "event");
    if (rc) { hipEventDestroy(e0); return rc; }
    rc = b->enter();
    if (!rc) rc = b->hip(hipEventRecord(e0, b->stream), "event record");
    if (!rc) rc = b->step_eager(nsteps);
    if (!rc) rc = b->hip(hipEventRecord(e1, b->stream), "event record");
    rc = b->leave(rc);
    if (!rc) rc = b->hip(hipEventSynchronize(e1), "event sync");
    float t = 0.f;
    if (!rc) rc = b->hip(hipEventElapsedTime(&t, e0, e1), "elapsed");
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    *ms = t;
    return rc;
}

int lbm_ms_batch_converge(lbm_ms_batch_t b, double tol, int64_t max_steps, int check_every,
                          int64_t* steps_taken, double* residual, int* status)
{
    if (!b || check_every <= 0 || max_steps < 0) return LBM_MS_E_ARG;
    for (auto* h : b->inst)
        if (!h->ready) return b->fail(LBM_MS_E_STATE, "init first");
    int rc = b->enter();
    if (rc) return rc;
    std::vector<int64_t> taken_k(b->count, 0);
    std::vector<double> r_k(b->count, INFINITY);
    std::vector<int> st_k(b->count, LBM_MS_E_NOT_CONVERGED);
    // fresh residual windows
    for (int k = 0; k < b->count && rc == LBM_MS_OK; ++k) {
        if (!b->active[k]) { st_k[k] = b->retired_status[k]; continue; }
        double v[6];
        rc = reduce_state(b->inst[k], 1, v);
        b->inst[k]->snap_step = b->inst[k]->steps;
    }
    int64_t taken = 0;
    bool changed = false;
    while (rc == LBM_MS_OK && taken < max_steps) {
        int n_active = 0;
        for (int k = 0; k < b->count; ++k) n_active += b->active[k];
        if (n_active == 0) break;
        if (changed) {
            rc = b->upload_active_tiles();
            if (rc == LBM_MS_OK) rc = b->upload_slots();
            if (rc) break;
            changed = false;
        }
        const int64_t n = std::min<int64_t>(check_every, max_steps - taken);
        rc = (b->use_graphs && n == check_every) ? b->step_graph((int)n) : b->step_eager(n);
        if (rc) break;
        taken += n;
        // every active instance's reduction in one pass over the batch, one wait, then the checks
        rc = b->check_all();
        if (rc) break;
        for (int k = 0; k < b->count; ++k) {
            if (!b->active[k]) continue;
            double r = 0;
            const int rk = residual_eval(b->inst[k], &r);
            taken_k[k] = taken;
            r_k[k] = r;
            if (rk == LBM_MS_E_HIP) {
                rc = rk;
                b->err = "instance " + std::to_string(k) + ": " + b->inst[k]->err;
                break;
            }
            if (rk != LBM_MS_OK || r < tol) {  // converged, or failed: leave the work list
                st_k[k] = rk;
                b->retired_status[k] = rk;
                b->active[k] = 0;
                changed = true;
            }
        }
    }
    // instances that left in the last check leave the work list now, so that later steps and
    // checks skip them as well
    if (changed && rc == LBM_MS_OK) {
        rc = b->upload_active_tiles();
        if (rc == LBM_MS_OK) rc = b->upload_slots();
    }
    if (steps_taken) std::memcpy(steps_taken, taken_k.data(), sizeof(int64_t) * b->count);
    if (residual) std::memcpy(residual, r_k.data(), sizeof(double) * b->count);
    if (status) std::memcpy(status, st_k.data(), sizeof(int) * b->count);
    if (rc == LBM_MS_OK) {
        for (int k = 0; k < b->count; ++k)
            if (st_k[k] != LBM_MS_OK) {
                rc = b->fail(st_k[k], "instance " + std::to_string(k) + ": " +
                                          lbm_ms_status_string(st_k[k]));
                break;
            }
    }
    return b->leave(rc);
}

int lbm_ms_batch_overpotential(lbm_ms_batch_t b, double* eta)
{
    if (!b || !eta) return LBM_MS_E_ARG;
    int rc = b->enter();
    for (int k = 0; k < b->count && rc == LBM_MS_OK; ++k) {
        rc = lbm_ms_overpotential(b->inst[k], &eta[k]);
        if (rc) b->err = "instance " + std::to_string(k) + ": " + b->inst[k]->err;
    }
    return b->leave(rc);
}

}  // extern "C"
