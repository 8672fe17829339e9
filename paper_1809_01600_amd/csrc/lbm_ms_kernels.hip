// HIP kernels (gfx950) of the LBM / Maxwell-Stefan time step and its reductions.
//
// Step kernels are pull-scheme and fused: each fluid node pulls its post-collision populations
// from the neighbours (bounce-back and the x-boundary rules applied on the way), forms the
// moments, takes the mole-fraction gradients from an LDS tile that also holds a one-node halo
// (recomputed from the halo nodes' own pulls), solves the Maxwell-Stefan system in FP64 for the
// relaxation times, collides and stores to the other buffer.  Populations of fluid nodes only
// are stored, one array per link with the two species of a node side by side ([link][fluid
// node][species]); fluid nodes are numbered strip by strip of 64 voxels in x in 2D (raster order
// within a strip) and, in 3D, column by column of 64 x 16 voxels, plane by plane, each plane's
// two x-edge lines first and then its rows in raster order.  A dense int32
// map gives each voxel's fluid index (-1 = solid), so solid voxels cost no population traffic
// while a wavefront's loads and stores stay contiguous along x.
#include <hip/hip_runtime.h>
#include <type_traits>

#include "lbm_ms_device.hpp"
#include "lbm_ms_kernels.hpp"

namespace lbmms {

// Source slots of a node from an LDS-staged copy of the index map.  The staged region covers the
// tile plus a two-node ring, so every source of a tile or halo node lies inside it.  sI points at
// NPL planes of RY x RX ints; the node sits at column cx, row cy of relative plane zr (plane slot
// (zr + 2) % NPL).  Lanes without a fluid node get zero slots (a harmless dummy gather).
template <class L, int RX, int RY, int NPL>
__device__ inline uint32_t lds_sources(const int* sI, int zr, int cx, int cy, int x, int nx, int i,
                                       int (&si)[L::Q])
{
    uint32_t nb = 0;
#pragma unroll
    for (int k = 0; k < L::Q; ++k) {
        const int ex = L::ex[k], ey = L::ey[k], ez = L::ez[k];
        if (k == 0) { si[k] = i; continue; }
        if ((ex == -1 && x == nx - 1) || (ex == 1 && x == 0)) { si[k] = BOUNDARY; continue; }
        const int slot = (zr - ez + 2 + NPL) % NPL;
        si[k] = sI[(slot * RY + (cy - ey)) * RX + (cx - ex)];
        nb |= axis_bit<L>(k, si[k]);
    }
    if (i < 0) {
#pragma unroll
        for (int k = 0; k < L::Q; ++k) si[k] = 0;
    }
    return nb;
}

// Halo ring position of thread t (t < 2 TX + 2 TY): tile-relative column hx and row hy.
template <int TX, int TY>
__device__ inline void halo_pos(int t, int& hx, int& hy)
{
    if (t < TX) { hx = t; hy = -1; }
    else if (t < 2 * TX) { hx = t - TX; hy = TY; }
    else if (t < 2 * TX + TY) { hx = -1; hy = t - 2 * TX; }
    else if (t < 2 * TX + 2 * TY) { hx = TX; hy = t - 2 * TX - TY; }
    else { hx = 0; hy = 0; }
}

// Periodic row of the staged region: gy = y0 - 2 + ry lies in [-2, ny + RY - 3] for a tile
// origin y0 in [0, ny), so one conditional wrap suffices once ny >= RY; smaller boxes (a
// workgroup-uniform branch) take the general remainder.  This keeps integer divisions, about
// twenty instructions each, out of the per-element staging loops.
template <int RY>
__device__ inline int wrap_row(int gy, int ny)
{
    if (ny >= RY) return gy < 0 ? gy + ny : (gy >= ny ? gy - ny : gy);
    return (gy % ny + ny) % ny;
}

// Stage the index map of plane z (periodic) for the region x in [x0-2, x0+TX+2), y in
// [y0-2, y0+TY+2) into dst; columns outside the box read -2.
template <int RX, int RY>
__device__ inline void stage_plane(const StepArgs& a, int x0, int y0, int z, int* dst)
{
    const long long zb = (long long)((z % a.nz + a.nz) % a.nz) * a.nx * a.ny;
    for (int t = threadIdx.x; t < RX * RY; t += blockDim.x) {
        const int rx = t % RX, ry = t / RX;
        const int gx = x0 - 2 + rx;
        const int gy = wrap_row<RY>(y0 - 2 + ry, a.ny);
        dst[t] = (gx >= 0 && gx < a.nx) ? gload<int>(a.idx, (unsigned)(zb + (long long)gy * a.nx + gx) * 4u) : -2;
    }
}

// stage_plane in two halves for a caller that overlaps the index loads with other work: the
// loads of this thread's share of plane z into registers, then their store into dst (NT threads).
template <int RX, int RY, int NT>
struct PlaneRegs {
    int v[(RX * RY + NT - 1) / NT];
};
template <int RX, int RY, int NT>
__device__ inline void stage_issue(const StepArgs& a, int x0, int y0, int z, PlaneRegs<RX, RY, NT>& r)
{
    // the box and the map read once, before the loads (read inside the conditional loads they
    // would be fetched again, with a wait, for every element)
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const int* idx = a.idx;
    const long long zb = (long long)((z % nz + nz) % nz) * nx * ny;
#pragma unroll
    for (int j = 0; j < (RX * RY + NT - 1) / NT; ++j) {
        const int t = threadIdx.x + j * NT;
        const int rx = t % RX, ry = t / RX;
        const int gx = x0 - 2 + rx;
        const int gy = wrap_row<RY>(y0 - 2 + ry, ny);
        r.v[j] = (t < RX * RY && gx >= 0 && gx < nx)
                     ? gload<int>(idx, (unsigned)(zb + (long long)gy * nx + gx) * 4u) : -2;
    }
}
template <int RX, int RY, int NT>
__device__ inline void stage_store(const PlaneRegs<RX, RY, NT>& r, int* dst)
{
#pragma unroll
    for (int j = 0; j < (RX * RY + NT - 1) / NT; ++j) {
        const int t = threadIdx.x + j * NT;
        if (t < RX * RY) dst[t] = r.v[j];
    }
}

// stage_plane of a 2D box in chunks of four ints: thread t stages chunk t (row t / (RX / 4), ints
// 4 (t % (RX / 4)) .. + 3 of it), with one 16-byte load where the chunk lies inside the box in x
// (the map's rows are only 4-byte aligned; gfx950 loads such a vector in one instruction) and
// element by element at the box's x faces; a quarter of the load instructions of stage_issue.
typedef int int4u __attribute__((ext_vector_type(4), aligned(4)));
template <int RX, int RY, int NT>
struct PlaneRegs4 {
    static constexpr int NC = RY * (RX / 4);  // chunks in the region
    int4u v[(NC + NT - 1) / NT];
};
template <int RX, int RY, int NT>
__device__ inline void stage_issue4(const StepArgs& a, int x0, int y0, PlaneRegs4<RX, RY, NT>& r,
                                    int z = 0)
{
    static_assert(RX % 4 == 0, "rows of whole chunks");
    constexpr int CR = RX / 4, NC = PlaneRegs4<RX, RY, NT>::NC;
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const int* idx = a.idx;
    const unsigned zb = (unsigned)((z % nz + nz) % nz) * (unsigned)(nx * ny);  // plane z, periodic
#pragma unroll
    for (int j = 0; j < (NC + NT - 1) / NT; ++j) {
        const int c = threadIdx.x + j * NT;
        const int ry = c / CR, gx = x0 - 2 + 4 * (c % CR);
        const int gy = wrap_row<RY>(y0 - 2 + ry, ny);
        const unsigned base = (zb + (unsigned)(gy * nx + gx)) * 4u;
        int4u v = {-2, -2, -2, -2};
        if (c < NC) {
            if (gx >= 0 && gx + 3 < nx) {
                v = *(const LBMMS_GLOBAL int4u*)((const LBMMS_GLOBAL char*)idx + base);
            } else {
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    if (gx + e >= 0 && gx + e < nx) v[e] = gload<int>(idx, base + 4u * (unsigned)e);
            }
        }
        r.v[j] = v;
    }
}
template <int RX, int RY, int NT>
__device__ inline void stage_store4(const PlaneRegs4<RX, RY, NT>& r, int* dst)
{
    constexpr int CR = RX / 4, NC = PlaneRegs4<RX, RY, NT>::NC;
#pragma unroll
    for (int j = 0; j < (NC + NT - 1) / NT; ++j) {
        const int c = threadIdx.x + j * NT;
        if (c < NC) *(int4*)(dst + (c / CR) * RX + 4 * (c % CR)) = make_int4(r.v[j].x, r.v[j].y, r.v[j].z, r.v[j].w);
    }
}

// The index maps of planes z0 - 2 .. z0 + 2 into ring slots (zr + 2) % NPL, every load issued
// before the first store (a loop of load, wait and store per element would take one memory round
// trip per element a thread stages).
template <int RX, int RY, int NT, int NPL>
__device__ inline void stage_ring(const StepArgs& a, int x0, int y0, int z0, int* sI)
{
    PlaneRegs<RX, RY, NT> r[5];
#pragma unroll
    for (int zr = -2; zr <= 2; ++zr) stage_issue<RX, RY, NT>(a, x0, y0, z0 + zr, r[zr + 2]);
#pragma unroll
    for (int zr = -2; zr <= 2; ++zr) stage_store<RX, RY, NT>(r[zr + 2], sI + ((zr + 2) % NPL) * RY * RX);
}

// The second half of staging a plane for the NODE shift, once stage_issue's index loads are in
// registers: the FP64 references c of its fluid nodes (all loads issued first), then the index
// map into dst and the references into sc ([species][RY * RX]).
template <int RX, int RY, int NT>
__device__ inline void stage_refs_store(const StepArgs& a, const PlaneRegs<RX, RY, NT>& r, int* dst,
                                        double* sc)
{
    constexpr int NR = (RX * RY + NT - 1) / NT;
    double c0[NR], c1[NR];
#pragma unroll
    for (int j = 0; j < NR; ++j) {
        const int i = r.v[j];
        c0[j] = i >= 0 ? gload<double>(a.xin, (unsigned)i * 8u) : 0.0;
        c1[j] = i >= 0 ? gload<double>(a.xin, (unsigned)(a.NF + i) * 8u) : 0.0;
    }
#pragma unroll
    for (int j = 0; j < NR; ++j) {
        const int t = threadIdx.x + j * NT;
        if (t < RX * RY) {
            dst[t] = r.v[j];
            sc[t] = c0[j];
            sc[RX * RY + t] = c1[j];
        }
    }
}

// stage_plane of a 2D box plus, for the NODE shift, the FP64 references c of every staged fluid
// node, in three rounds: all index loads, then all reference loads, then the stores (NT threads).
template <int RX, int RY, int NT>
__device__ inline void stage_plane_refs_pipelined(const StepArgs& a, int x0, int y0, int* dst, double* sc)
{
    constexpr int NR = (RX * RY + NT - 1) / NT;
    PlaneRegs<RX, RY, NT> r;
    stage_issue<RX, RY, NT>(a, x0, y0, 0, r);
    double c0[NR], c1[NR];
#pragma unroll
    for (int j = 0; j < NR; ++j) {
        const int i = r.v[j];
        c0[j] = i >= 0 ? gload<double>(a.xin, (unsigned)i * 8u) : 0.0;
        c1[j] = i >= 0 ? gload<double>(a.xin, (unsigned)(a.NF + i) * 8u) : 0.0;
    }
#pragma unroll
    for (int j = 0; j < NR; ++j) {
        const int t = threadIdx.x + j * NT;
        if (t < RX * RY) {
            dst[t] = r.v[j];
            sc[t] = c0[j];
            sc[RX * RY + t] = c1[j];
        }
    }
}

// Pull of one node of a 2D tile: NODE-shift references from the staged region, else the plain
// gather.  (cx, cy): the node's position in the staged region.
template <class L, int P, bool NS, int RX, int RY>
__device__ inline void gather2d(const StepArgs& a, int i, const int (&si)[L::Q], bool inlet,
                                bool outlet, typename Codec<P>::CT (&f)[2][L::Q], double& X0,
                                double& X1, const double* sc, int cx, int cy)
{
    if constexpr (NS)
        gather_ns<L, P>(a, i, si, inlet, outlet, f, X0, X1, RefLds<RX, RY>{sc, cy * RX + cx});
    else
        gather<L, P, false>(a, i, si, inlet, outlet, f, X0, X1);
}

// ---------------------------------------------------------------------------------------------
// 2D (D2Q9): a work list of 64 x TY tiles.  Each tile record names its instance (one problem of
// a batch), its origin, and two entry lists built on the host: the tile's fluid nodes and the
// fluid nodes outside them whose moments the tile's gradients read (the halo).  Entries are LDS
// coordinates (cx, cy) of the (TX + 2) x (TY + 2) moment tile, packed as cy << 8 | cx.  Every
// lane works on a fluid node; two memory round trips (staged index map, then all population
// loads of the tile and its halo at once).  Workgroup = 32 TY lanes and a lane holds at most one
// own node: the host splits a tile with more fluid nodes into parts, each listing the others'
// nodes it needs as halo.  One node per lane keeps the register count low enough for eight
// waves per SIMD.
// ---------------------------------------------------------------------------------------------
// The work of one tile once its index map is staged in sI: the pulls of its own nodes and of its
// halo, the moments into sX, one barrier, then gradients, the Maxwell-Stefan solve, the collision
// and the store.  t1 = (own offset, own count, halo offset, halo count) in ent; pe0 / pe2 = this
// lane's first own and halo entries.  BND: the tile or its halo touches an x face.
template <class L, int P, bool NS, int TY, int TYR, bool BND>
__device__ inline void tile_work(const StepArgs& a, int x0, int y0, const int4& t1, unsigned pe0,
                                 unsigned pe2, const unsigned* __restrict__ ent, const int* sI,
                                 double (&sX)[2][TYR + 2][64 + 2], const double* sC)
{
    using CT = typename Codec<P>::CT;
    constexpr int TX = 64, RX = TX + 4, RY = TYR + 4, BS = 32 * TY;
    (void)y0;

    // the lane's own node (at most one: the host splits denser tiles) and its first halo entry:
    // all loads issued together
    CT f[2][L::Q];
    double X0 = 0.0, X1 = 0.0;
    const int cxo = pe0 & 255u, cyo = pe0 >> 8;
    const int io = threadIdx.x < (unsigned)t1.y ? sI[(cyo + 1) * RX + cxo + 1] : -1;
    uint32_t nbo;
    {
        const int x = x0 + cxo - 1;
        int si[L::Q];
        nbo = lds_sources<L, RX, RY, 1>(sI, -2, cxo + 1, cyo + 1, x, a.nx, io, si);
        gather2d<L, P, NS, RX, RY>(a, io < 0 ? 0 : io, si, io >= 0 && BND && x == 0, io >= 0 && BND && x == a.nx - 1,
                                f, X0, X1, sC, cxo + 1, cyo + 1);
    }
    if ((threadIdx.x & ~63u) < (unsigned)t1.w) {  // wave-uniform: this wave holds halo lanes
        const int cx = pe2 & 255u, cy = pe2 >> 8;
        const bool job = threadIdx.x < (unsigned)t1.w;
        const int hi = job ? sI[(cy + 1) * RX + cx + 1] : -1;
        const int x = x0 + cx - 1;
        int si[L::Q];
        lds_sources<L, RX, RY, 1>(sI, -2, cx + 1, cy + 1, x, a.nx, hi, si);
        CT hf[2][L::Q];
        double h0, h1;
        gather2d<L, P, NS, RX, RY>(a, hi < 0 ? 0 : hi, si, hi >= 0 && BND && x == 0, hi >= 0 && BND && x == a.nx - 1,
                                hf, h0, h1, sC, cx + 1, cy + 1);
        if (job) {
            sX[0][cy][cx] = h0;
            sX[1][cy][cx] = h1;
        }
    }
    // remaining halo entries (a tile that wraps onto itself in y, or one part of a split tile)
    for (int e = threadIdx.x + BS; e < t1.w; e += BS) {
        const unsigned pw = gload<unsigned>(ent, (unsigned)(t1.z + e) * 4u);
        const int cx = pw & 255u, cy = pw >> 8;
        const int hi = sI[(cy + 1) * RX + cx + 1];
        const int x = x0 + cx - 1;
        int si[L::Q];
        lds_sources<L, RX, RY, 1>(sI, -2, cx + 1, cy + 1, x, a.nx, hi, si);
        CT hf[2][L::Q];
        double h0, h1;
        gather2d<L, P, NS, RX, RY>(a, hi, si, BND && x == 0, BND && x == a.nx - 1, hf, h0, h1, sC, cx + 1, cy + 1);
        sX[0][cy][cx] = h0;
        sX[1][cy][cx] = h1;
    }
    if (io >= 0) {
        sX[0][cyo][cxo] = X0;
        sX[1][cyo][cxo] = X1;
    }
    __syncthreads();

    if (io < 0) return;
    const int cx = cxo, cy = cyo;
    double g0[3], g1[3];
    const bool xp = nbo & NB_XP, xm = nbo & NB_XM, yp = nbo & NB_YP, ym = nbo & NB_YM;
    g0[0] = grad1(xp, xm, sX[0][cy][cx + 1], X0, sX[0][cy][cx - 1]);
    g1[0] = grad1(xp, xm, sX[1][cy][cx + 1], X1, sX[1][cy][cx - 1]);
    g0[1] = grad1(yp, ym, sX[0][cy + 1][cx], X0, sX[0][cy - 1][cx]);
    g1[1] = grad1(yp, ym, sX[1][cy + 1][cx], X1, sX[1][cy - 1][cx]);
    g0[2] = g1[2] = 0.0;
    double om0, om1;
    bool hit;
    ms_relax<2>(a, X0, X1, g0, g1, BND && x0 + cx - 1 == a.nx - 1, om0, om1, hit);
    if (hit) gstore<unsigned>(a.flags, 0u, 1u);
    const bool src = x0 + cx - 1 >= a.src_x0;
    collide_store<L, P, NS>(a, io, f, X0, X1, om0, om1, src ? a.S0 : 0.0, src ? a.S1 : 0.0);
}

// Global-shift FP32 and 16-bit instantiations fit in 64 VGPRs: ask for eight waves per SIMD for
// every tile height.  (HIP passes the second launch-bounds argument to the compiler as the
// minimum number of waves per SIMD, not as CUDA's workgroups per multiprocessor.)
template <int P, bool NS>
constexpr int step2d_min_waves() { return (P != P_F64 && !NS) ? 8 : 1; }

// TYR: rows of the staged region and moment tile.  TYR = TY for fixed 64 x TY tiles; a larger
// TYR for packed tiles, which the host grows row by row up to TYR rows or 32 TY fluid nodes.
template <class L, int P, bool NS, int TY, int TYR>
__global__ __launch_bounds__(32 * TY, (step2d_min_waves<P, NS>())) void k_step2d(const StepArgs* __restrict__ insts,
                                                    const int4* __restrict__ tiles,
                                                    const unsigned* __restrict__ ent)
{
    using CT = typename Codec<P>::CT;
    constexpr int TX = 64, RX = TX + 4, RY = TYR + 4, BS = 32 * TY;
    __shared__ __align__(16) int sI[RY * RX];
    __shared__ double sX[2][TYR + 2][TX + 2];
    __shared__ double sC[NS ? 2 * RY * RX : 1];  // NODE shift: staged references

    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const unsigned tb = (unsigned)tile * 32u;
    const int4 t0 = make_int4(gload<int>(tiles, tb), gload<int>(tiles, tb + 4u),
                              gload<int>(tiles, tb + 8u), 0);  // x0, y0, instance
    const int4 t1 = make_int4(gload<int>(tiles, tb + 16u), gload<int>(tiles, tb + 20u),
                              gload<int>(tiles, tb + 24u), gload<int>(tiles, tb + 28u));  // own/halo offsets, counts
    const StepArgs& a = insts[t0.z];
    const int x0 = t0.x, y0 = t0.y;
    // entry lists first (they depend only on the tile record), then the staged index map
    const unsigned dummy = (1u << 8) | 1u;
    const unsigned pe0 = threadIdx.x < (unsigned)t1.y ? gload<unsigned>(ent, (unsigned)(t1.x + threadIdx.x) * 4u) : dummy;
    const unsigned pe2 = threadIdx.x < (unsigned)t1.w ? gload<unsigned>(ent, (unsigned)(t1.z + threadIdx.x) * 4u) : dummy;
    // Every staging load of a thread is issued before its first store (a loop of load, wait and
    // store per element costs a memory round trip per element): the global shift stages 16-byte
    // chunks; the NODE shift stages elements, and its references, which need the indices, follow
    // in a second round (chunks measured slower there).
    if constexpr (NS) {
        stage_plane_refs_pipelined<RX, RY, BS>(a, x0, y0, sI, sC);
    } else {
        PlaneRegs4<RX, RY, BS> stg;
        stage_issue4<RX, RY, BS>(a, x0, y0, stg);
        stage_store4<RX, RY, BS>(stg, sI);
    }
    __syncthreads();

    // Tiles whose nodes and halo touch neither the inlet column nor the outlet column run a copy
    // of the rest with the boundary rules compiled out (a workgroup-uniform branch).
    const bool edge = x0 == 0 || x0 + TX + 1 >= a.nx;
    if (edge)
        tile_work<L, P, NS, TY, TYR, true>(a, x0, y0, t1, pe0, pe2, ent, sI, sX, sC);
    else
        tile_work<L, P, NS, TY, TYR, false>(a, x0, y0, t1, pe0, pe2, ent, sI, sX, sC);
}

// stage_plane for plane z plus, for the NODE shift, the FP64 references of its fluid nodes into
// the matching slot of the reference ring ([species][RY * RX] per slot).
template <int RX, int RY>
__device__ inline void stage_plane_refs3d(const StepArgs& a, int x0, int y0, int z, int* dst,
                                          double* sc)
{
    const long long zb = (long long)((z % a.nz + a.nz) % a.nz) * a.nx * a.ny;
    for (int t = threadIdx.x; t < RX * RY; t += blockDim.x) {
        const int rx = t % RX, ry = t / RX;
        const int gx = x0 - 2 + rx;
        const int gy = wrap_row<RY>(y0 - 2 + ry, a.ny);
        const int i = (gx >= 0 && gx < a.nx) ? gload<int>(a.idx, (unsigned)(zb + (long long)gy * a.nx + gx) * 4u) : -2;
        dst[t] = i;
        sc[t] = i >= 0 ? gload<double>(a.xin, (unsigned)i * 8u) : 0.0;
        sc[RX * RY + t] = i >= 0 ? gload<double>(a.xin, (unsigned)(a.NF + i) * 8u) : 0.0;
    }
}

// Pull of one node of a 3D tile: NODE-shift references from the staged ring, else the plain
// gather.  (cx, cy): the node's position in the staged plane, zr its relative plane.
template <class L, int P, bool NS, int RX, int RY, int NPL>
__device__ inline void gather3d(const StepArgs& a, int i, const int (&si)[L::Q], bool inlet,
                                bool outlet, typename Codec<P>::CT (&f)[2][L::Q], double& X0,
                                double& X1, const double* sc, int zr, int cx, int cy)
{
    if constexpr (NS)
        gather_ns<L, P>(a, i, si, inlet, outlet, f, X0, X1, RefLds3<RX, RY, NPL>{sc, zr, cy * RX + cx});
    else
        gather<L, P, false>(a, i, si, inlet, outlet, f, X0, X1);
}

// ---------------------------------------------------------------------------------------------
// 3D (D3Q19, D3Q7): one workgroup = 64 x TY column tile marching through CZ planes.  The index map is
// staged in a 5-plane LDS ring one plane ahead; x/y gradients come from a 3-slot LDS ring of
// plane moments (tile + halo ring), z gradients from the column's own rolling registers.  One
// barrier per plane.
// ---------------------------------------------------------------------------------------------
// D3Q7 with global-shift storage fits 128 VGPRs: ask for four waves per SIMD (the second
// launch-bounds argument counts waves per SIMD)
template <class L, int P, bool NS, int TY>
constexpr int step3d_min_waves() { return (std::is_same<L, D3Q7>::value && !NS && P != P_F64 && TY == 8) ? 4 : 1; }

template <class L, int P, bool NS, int TY, int CZ>
__global__ __launch_bounds__(64 * TY, (step3d_min_waves<L, P, NS, TY>())) void k_step3d(StepArgs a)
{
    using CT = typename Codec<P>::CT;
    constexpr int TX = 64, RX = TX + 4, RY = TY + 4, NPL = 5;
    constexpr int NHALO = 2 * TX + 2 * TY;
    constexpr int HWAVES = (NHALO + 63) / 64;
    __shared__ int sI[NPL * RY * RX];
    __shared__ double sX[3][2][TY + 2][TX + 2];
    __shared__ double sC[NS ? NPL * 2 * RY * RX : 1];  // NODE shift: staged reference ring

    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int bx = tile % a.tiles_x;
    const int rest = tile / a.tiles_x;
    const int by = rest % a.tiles_y;
    const int bz = rest / a.tiles_y;
    const int x0 = bx * TX, y0 = by * TY, z0 = bz * CZ;
    const int lx = threadIdx.x & (TX - 1);
    const int ly = threadIdx.x / TX;
    const int x = x0 + lx;
    const bool own = (x < a.nx) && (y0 + ly < a.ny);
    const bool in_x = x < a.nx;
    int hx = 0, hy = 0;
    halo_pos<TX, TY>(threadIdx.x, hx, hy);
    const int hgx = x0 + hx;
    const bool hjob = threadIdx.x < NHALO && hgx >= 0 && hgx < a.nx;
    auto stage = [&](int zrel) {  // plane z0 + zrel into ring slot (zrel + 2) % NPL
        const int slot = (zrel + 2) % NPL;
        if constexpr (NS)
            stage_plane_refs3d<RX, RY>(a, x0, y0, z0 + zrel, sI + slot * RY * RX, sC + slot * 2 * RY * RX);
        else
            stage_plane<RX, RY>(a, x0, y0, z0 + zrel, sI + slot * RY * RX);
    };

    // planes z0-2 .. z0+2 (relative -2 .. 2) into the ring
    if constexpr (NS) {
        for (int zr = -2; zr <= 2; ++zr)
            stage(zr);
    } else {
        stage_ring<RX, RY, 64 * TY, NPL>(a, x0, y0, z0, sI);
    }
    __syncthreads();

    // plane z0-1: moments only (z gradient of plane z0); plane z0: populations and moments
    double Xm0, Xm1, Xc0, Xc1;
    CT fc[2][L::Q];
    int ic;
    uint32_t nbc;
    {
        const int im = sI[((1) * RY + ly + 2) * RX + lx + 2];
        int si[L::Q];
        lds_sources<L, RX, RY, NPL>(sI, -1, lx + 2, ly + 2, x, a.nx, in_x ? im : -1, si);
        CT tf[2][L::Q];
        gather3d<L, P, NS, RX, RY, NPL>(a, (in_x && im >= 0) ? im : 0, si, x == 0, x == a.nx - 1, tf, Xm0, Xm1,
                                     sC, -1, lx + 2, ly + 2);
        if (!(in_x && im >= 0)) Xm0 = Xm1 = 0.0;
        ic = in_x ? sI[((2) * RY + ly + 2) * RX + lx + 2] : -1;
        nbc = lds_sources<L, RX, RY, NPL>(sI, 0, lx + 2, ly + 2, x, a.nx, ic, si);
        gather3d<L, P, NS, RX, RY, NPL>(a, ic < 0 ? 0 : ic, si, x == 0, x == a.nx - 1, fc, Xc0, Xc1, sC, 0,
                                     lx + 2, ly + 2);
        if (ic < 0) Xc0 = Xc1 = 0.0;
        double h0 = 0.0, h1 = 0.0;
        if (threadIdx.x < HWAVES * 64) {
            const int hi = hjob ? sI[((2) * RY + hy + 2) * RX + hx + 2] : -1;
            int hsi[L::Q];
            lds_sources<L, RX, RY, NPL>(sI, 0, hx + 2, hy + 2, hgx, a.nx, hi, hsi);
            CT hf[2][L::Q];
            gather3d<L, P, NS, RX, RY, NPL>(a, hi < 0 ? 0 : hi, hsi, hjob && hgx == 0, hjob && hgx == a.nx - 1,
                                         hf, h0, h1, sC, 0, hx + 2, hy + 2);
            if (hi < 0) h0 = h1 = 0.0;
        }
        sX[0][0][ly + 1][lx + 1] = Xc0;
        sX[0][1][ly + 1][lx + 1] = Xc1;
        if (threadIdx.x < NHALO) {
            sX[0][0][hy + 1][hx + 1] = h0;
            sX[0][1][hy + 1][hx + 1] = h1;
        }
    }
    __syncthreads();  // the ring slot of plane z0-2 is free from here on

    // The memory round trips of an iteration overlap: the index loads of the plane staged for
    // later and the population loads of the own column and of the halo are all issued before any
    // of them is used, and the staged plane is stored to LDS last (its slot is not read in this
    // iteration, but the compiler cannot tell, so an early store would hold the pull's LDS reads
    // behind the index loads).  The NODE shift then loads the staged plane's references, which
    // need the indices, in one more round trip before the store.  FP64 keeps the halo after the
    // own column: its registers are already full.
    constexpr bool OVERLAP = !NS;
    constexpr bool MERGE_HALO = !NS && P != P_F64;
    // The in-plane half of the Maxwell-Stefan work (x/y gradients, [B], 1/det) can run while the
    // next plane's populations are in flight.  That holds 12 more registers across the wait:
    // D3Q19 has room below 256 (3% faster), while D3Q7 would cross 128 and lose a wave per SIMD
    // (26% slower), so D3Q7 keeps the work after the barrier.
    constexpr bool HOIST = MERGE_HALO && std::is_same<L, D3Q19>::value;
    using raw = typename Codec<P>::raw;
    for (int it = 0; it < CZ; ++it) {
        const int zi = z0 + it;
        if (zi >= a.nz) break;  // uniform across the workgroup
        // stage plane it+3 (read by the next iteration's pull)
        // (the NODE shift also needs the plane's references, loaded once the indices are in)
        PlaneRegs<RX, RY, 64 * TY> stg;
        stage_issue<RX, RY, 64 * TY>(a, x0, y0, z0 + it + 3, stg);
        // pull plane it+1: own column (populations kept) and, if the next plane is output, its halo
        const int zr = it + 1;
        const int pslot = (zr + 2) % NPL;
        const int in_ = in_x ? sI[(pslot * RY + ly + 2) * RX + lx + 2] : -1;
        int si[L::Q];
        const uint32_t nbn = lds_sources<L, RX, RY, NPL>(sI, zr, lx + 2, ly + 2, x, a.nx, in_, si);
        const bool need_next = (it + 1 < CZ) && (zi + 1 < a.nz);
        const bool hwave = need_next && threadIdx.x < HWAVES * 64;  // uniform per wave
        const int hi = (hwave && hjob) ? sI[(pslot * RY + hy + 2) * RX + hx + 2] : -1;
        CT fn[2][L::Q];
        double Xp0, Xp1, h0 = 0.0, h1 = 0.0;
        // HOIST: the in-plane gradients and the Maxwell-Stefan matrix of the node collided in
        // this iteration, taken while the loads are in flight; they read only plane it's
        // moments, written before the previous barrier
        double hg0[3], hg1[3];
        MsMat hms;
        if constexpr (MERGE_HALO) {
            raw rn[2][L::Q], rh[2][L::Q];
            gather_issue<L, P>(a, in_ < 0 ? 0 : in_, si, x == 0, x == a.nx - 1, rn);
            if (hwave) {
                int hsi[L::Q];
                lds_sources<L, RX, RY, NPL>(sI, zr, hx + 2, hy + 2, hgx, a.nx, hi, hsi);
                gather_issue<L, P>(a, hi < 0 ? 0 : hi, hsi, hjob && hgx == 0, hjob && hgx == a.nx - 1, rh);
            }
            if constexpr (HOIST) {
                const int s = it % 3;
                const int cx = lx + 1, cy = ly + 1;
                const bool xp = nbc & NB_XP, xm = nbc & NB_XM, yp = nbc & NB_YP, ym = nbc & NB_YM;
                hg0[0] = grad1(xp, xm, sX[s][0][cy][cx + 1], Xc0, sX[s][0][cy][cx - 1]);
                hg1[0] = grad1(xp, xm, sX[s][1][cy][cx + 1], Xc1, sX[s][1][cy][cx - 1]);
                hg0[1] = grad1(yp, ym, sX[s][0][cy + 1][cx], Xc0, sX[s][0][cy - 1][cx]);
                hg1[1] = grad1(yp, ym, sX[s][1][cy + 1][cx], Xc1, sX[s][1][cy - 1][cx]);
                hms = ms_matrix<true>(a, Xc0, Xc1);
            }
            gather_finish<L, P>(a, rn, x == 0, x == a.nx - 1, fn, Xp0, Xp1);
            if (hwave) {
                CT hf[2][L::Q];
                gather_finish<L, P>(a, rh, hjob && hgx == 0, hjob && hgx == a.nx - 1, hf, h0, h1);
            }
        } else {
            gather3d<L, P, NS, RX, RY, NPL>(a, in_ < 0 ? 0 : in_, si, x == 0, x == a.nx - 1, fn, Xp0, Xp1, sC,
                                         zr, lx + 2, ly + 2);
            if (hwave) {
                int hsi[L::Q];
                lds_sources<L, RX, RY, NPL>(sI, zr, hx + 2, hy + 2, hgx, a.nx, hi, hsi);
                CT hf[2][L::Q];
                gather3d<L, P, NS, RX, RY, NPL>(a, hi < 0 ? 0 : hi, hsi, hjob && hgx == 0,
                                             hjob && hgx == a.nx - 1, hf, h0, h1, sC, zr, hx + 2, hy + 2);
            }
        }
        if (in_ < 0) Xp0 = Xp1 = 0.0;
        if (hi < 0) h0 = h1 = 0.0;
        const int s_next = (it + 1) % 3;
        if (need_next) {
            sX[s_next][0][ly + 1][lx + 1] = Xp0;
            sX[s_next][1][ly + 1][lx + 1] = Xp1;
            if (threadIdx.x < NHALO) {
                sX[s_next][0][hy + 1][hx + 1] = h0;
                sX[s_next][1][hy + 1][hx + 1] = h1;
            }
        }
        if constexpr (OVERLAP)
            stage_store<RX, RY, 64 * TY>(stg, sI + (it + 5) % NPL * RY * RX);
        else
            stage_refs_store<RX, RY, 64 * TY>(a, stg, sI + (it + 5) % NPL * RY * RX,
                                              sC + (it + 5) % NPL * 2 * RY * RX);
        __syncthreads();
        if (own && ic >= 0) {
            const bool zpf = nbc & NB_ZP, zmf = nbc & NB_ZM;
            double om0, om1;
            bool hit;
            if constexpr (HOIST) {
                hg0[2] = grad1(zpf, zmf, Xp0, Xc0, Xm0);
                hg1[2] = grad1(zpf, zmf, Xp1, Xc1, Xm1);
                ms_relax<3, true>(a, Xc0, Xc1, hms, hg0, hg1, x == a.nx - 1, om0, om1, hit);
            } else {
                const int s = it % 3;
                const int cx = lx + 1, cy = ly + 1;
                double g0[3], g1[3];
                const bool xp = nbc & NB_XP, xm = nbc & NB_XM, yp = nbc & NB_YP, ym = nbc & NB_YM;
                g0[0] = grad1(xp, xm, sX[s][0][cy][cx + 1], Xc0, sX[s][0][cy][cx - 1]);
                g1[0] = grad1(xp, xm, sX[s][1][cy][cx + 1], Xc1, sX[s][1][cy][cx - 1]);
                g0[1] = grad1(yp, ym, sX[s][0][cy + 1][cx], Xc0, sX[s][0][cy - 1][cx]);
                g1[1] = grad1(yp, ym, sX[s][1][cy + 1][cx], Xc1, sX[s][1][cy - 1][cx]);
                g0[2] = grad1(zpf, zmf, Xp0, Xc0, Xm0);
                g1[2] = grad1(zpf, zmf, Xp1, Xc1, Xm1);
                ms_relax<3>(a, Xc0, Xc1, g0, g1, x == a.nx - 1, om0, om1, hit);
            }
            if (hit) gstore<unsigned>(a.flags, 0u, 1u);
            const bool src = x >= a.src_x0;
            collide_store<L, P, NS>(a, ic, fc, Xc0, Xc1, om0, om1, src ? a.S0 : 0.0, src ? a.S1 : 0.0);
        }
        Xm0 = Xc0; Xm1 = Xc1;
        Xc0 = Xp0; Xc1 = Xp1;
        ic = in_;
        nbc = nbn;
#pragma unroll
        for (int k = 0; k < L::Q; ++k) {
            fc[0][k] = fn[0][k];
            fc[1][k] = fn[1][k];
        }
    }
}

// ---------------------------------------------------------------------------------------------
// 3D over fluid-compacted planes (global-shift storage, 32- and 16-bit populations).  A workgroup
// owns a column of 64 x TY voxels (TY = 12 or 16) and marches CZ planes like k_step3d, but its
// 512 lanes take the fluid voxels of each plane in order, from a per-(column, plane) list of
// in-column positions built on the host, instead of one voxel each.  In a porous block about half
// the voxels are solid, so a plane of a 64 x 16 column fills about as many lanes as a 64 x 8
// plane leaves idle, and each wave's loads and FP64 solves carry twice the nodes.
//
// A plane with more fluid voxels than lanes hands the rest to a second pass: moments only before
// the barrier (the z gradients of the plane below need them), pulled again and collided after it.
// A lane's voxel moves from plane to plane, so z gradients come from the moment ring in LDS, four
// planes deep (below, own, above, and the one the next iteration writes), and the index ring
// holds six planes (a second-pass pull after the barrier still reads the planes around its own
// while the next iteration stages a new one).
// ---------------------------------------------------------------------------------------------
template <class L, int P, int TY, int CZ>
__global__ __launch_bounds__(512, 1) void k_step3dc(StepArgs a, const unsigned* __restrict__ coff,
                                                    const unsigned short* __restrict__ cpos)
{
    using CT = typename Codec<P>::CT;
    using raw = typename Codec<P>::raw;
    constexpr int NT = 512, TX = 64, RX = TX + 4, RY = TY + 4, NPL = 6;
    constexpr int NHALO = 2 * TX + 2 * TY;
    constexpr int HWAVES = (NHALO + 63) / 64;
    static_assert(TX * TY <= 2 * NT, "at most two passes per plane");
    __shared__ __align__(16) int sI[NPL * RY * RX];
    __shared__ double sX[4][2][TY + 2][TX + 2];  // moment ring: relative plane r in slot (r + 1) & 3

    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int bx = tile % a.tiles_x;
    const int rest = tile / a.tiles_x;
    const int by = rest % a.tiles_y;
    const int bz = rest / a.tiles_y;
    const int x0 = bx * TX, y0 = by * TY, z0 = bz * CZ;
    // plane offsets of this column: plane z holds positions [col[z], col[z + 1]) of cpos
    const unsigned* col = coff + (size_t)(bx + a.tiles_x * by) * a.nz;
    const int l = threadIdx.x;
    int hx = 0, hy = 0;
    halo_pos<TX, TY>(l, hx, hy);
    // The lists hold the column's rows inside the box only, so the row above a column cut short
    // by the box edge (y0 + TY > ny) belongs to the halo: that row of the staged region wraps to
    // y = 0, and its moments go where the column's last row looks for its +y neighbour.
    const int rows = a.ny - y0 < TY ? a.ny - y0 : TY;
    if (hy == TY) hy = rows;
    const int hgx = x0 + hx;
    const bool hjob = l < NHALO && hgx >= 0 && hgx < a.nx && hy <= rows;
    auto plane_of = [&](int r, unsigned& start, int& count) {  // list of relative plane r
        const int zw = ((z0 + r) % a.nz + a.nz) % a.nz;
        start = col[zw];
        count = (int)(col[zw + 1] - start);
    };
    auto index_at = [&](int r, int cx, int cy) { return sI[(((r + 2) % NPL) * RY + cy + 2) * RX + cx + 2]; };
    // moments of the fluid voxel at (cx, cy) of relative plane r into the ring
    auto moments_to_ring = [&](int r, int p) {
        const int cx = p & 63, cy = p >> 6, x = x0 + cx;
        const int i = index_at(r, cx, cy);
        int si[L::Q];
        lds_sources<L, RX, RY, NPL>(sI, r, cx + 2, cy + 2, x, a.nx, i, si);
        CT f[2][L::Q];
        double X0, X1;
        gather<L, P, false>(a, i, si, x == 0, x == a.nx - 1, f, X0, X1);
        sX[(r + 1) & 3][0][cy + 1][cx + 1] = X0;
        sX[(r + 1) & 3][1][cy + 1][cx + 1] = X1;
    };
    // Eq. 24-25 from the ring: x, y gradients in the node's plane r, z from the planes around it
    auto relax = [&](int r, int cx, int cy, uint32_t nb, double X0, double X1, bool outlet,
                     double& om0, double& om1) {
        const int s = (r + 1) & 3, su = (r + 2) & 3, sd = r & 3;
        const int px = cx + 1, py = cy + 1;
        double g0[3], g1[3];
        const bool xp = nb & NB_XP, xm = nb & NB_XM, yp = nb & NB_YP, ym = nb & NB_YM;
        const bool zp = nb & NB_ZP, zm = nb & NB_ZM;
        g0[0] = grad1(xp, xm, sX[s][0][py][px + 1], X0, sX[s][0][py][px - 1]);
        g1[0] = grad1(xp, xm, sX[s][1][py][px + 1], X1, sX[s][1][py][px - 1]);
        g0[1] = grad1(yp, ym, sX[s][0][py + 1][px], X0, sX[s][0][py - 1][px]);
        g1[1] = grad1(yp, ym, sX[s][1][py + 1][px], X1, sX[s][1][py - 1][px]);
        g0[2] = grad1(zp, zm, sX[su][0][py][px], X0, sX[sd][0][py][px]);
        g1[2] = grad1(zp, zm, sX[su][1][py][px], X1, sX[sd][1][py][px]);
        bool hit;
        ms_relax<3>(a, X0, X1, g0, g1, outlet, om0, om1, hit);
        if (hit) gstore<unsigned>(a.flags, 0u, 1u);
    };

    // D3Q19 stages the index map in 16-byte chunks (stage_issue4: FP32 0.638 -> 0.604 ms on the
    // 256^3 block); D3Q7, whose pull is a third as long, element by element (0.371 against 0.381)
    constexpr bool CHUNKS = std::is_same<L, D3Q19>::value;
    using Stage = typename std::conditional<CHUNKS, PlaneRegs4<RX, RY, NT>, PlaneRegs<RX, RY, NT>>::type;
    auto stage_issue_z = [&](Stage& r, int z) {
        if constexpr (CHUNKS) stage_issue4<RX, RY, NT>(a, x0, y0, r, z);
        else stage_issue<RX, RY, NT>(a, x0, y0, z, r);
    };
    auto stage_store_slot = [&](const Stage& r, int* dst) {
        if constexpr (CHUNKS) stage_store4<RX, RY, NT>(r, dst);
        else stage_store<RX, RY, NT>(r, dst);
    };
    {  // planes z0-2 .. z0+2 into ring slots (zr + 2) % NPL, every load issued first
        Stage r5[5];
#pragma unroll
        for (int zr = -2; zr <= 2; ++zr) stage_issue_z(r5[zr + 2], z0 + zr);
#pragma unroll
        for (int zr = -2; zr <= 2; ++zr) stage_store_slot(r5[zr + 2], sI + ((zr + 2) % NPL) * RY * RX);
    }
    __syncthreads();

    // plane z0-1: moments of every fluid voxel (z gradients of plane z0)
    unsigned st;
    int cnt;
    plane_of(-1, st, cnt);
    for (int k = l; k < cnt; k += NT) moments_to_ring(-1, cpos[st + k]);
    // plane z0: the first pass keeps its populations, a second pass and the halo ring give moments
    CT fc[2][L::Q];
    int ic = -1, pc = 0;
    uint32_t nbc = 0;
    double Xc0 = 0.0, Xc1 = 0.0;
    plane_of(0, st, cnt);
    int cnt_c = cnt;
    unsigned st_c = st;
    if (l < cnt) {
        pc = cpos[st + l];
        const int cx = pc & 63, cy = pc >> 6, x = x0 + cx;
        ic = index_at(0, cx, cy);
        int si[L::Q];
        nbc = lds_sources<L, RX, RY, NPL>(sI, 0, cx + 2, cy + 2, x, a.nx, ic, si);
        gather<L, P, false>(a, ic, si, x == 0, x == a.nx - 1, fc, Xc0, Xc1);
        sX[1][0][cy + 1][cx + 1] = Xc0;
        sX[1][1][cy + 1][cx + 1] = Xc1;
    }
    for (int k = l + NT; k < cnt; k += NT) moments_to_ring(0, cpos[st + k]);
    // the list of plane z0+1 and this lane's first-pass position in it, one plane ahead of use
    unsigned st_n;
    int cnt_n;
    plane_of(1, st_n, cnt_n);
    int p_n = l < cnt_n ? cpos[st_n + l] : 0;
    if (l < HWAVES * 64) {
        const int hi = hjob ? index_at(0, hx, hy) : -1;
        int hsi[L::Q];
        lds_sources<L, RX, RY, NPL>(sI, 0, hx + 2, hy + 2, hgx, a.nx, hi, hsi);
        CT hf[2][L::Q];
        double h0, h1;
        gather<L, P, false>(a, hi < 0 ? 0 : hi, hsi, hjob && hgx == 0, hjob && hgx == a.nx - 1, hf, h0, h1);
        if (l < NHALO) {
            sX[1][0][hy + 1][hx + 1] = hi < 0 ? 0.0 : h0;
            sX[1][1][hy + 1][hx + 1] = hi < 0 ? 0.0 : h1;
        }
    }
    __syncthreads();

    for (int it = 0; it < CZ; ++it) {
        const int zi = z0 + it;
        if (zi >= a.nz) break;  // uniform across the workgroup
        Stage stg;
        stage_issue_z(stg, z0 + it + 3);
        const int r = it + 1;
        const bool need_next = (it + 1 < CZ) && (zi + 1 < a.nz);
        st = st_n;
        cnt = cnt_n;
        const int pn = p_n;
        plane_of(r + 1, st_n, cnt_n);
        p_n = l < cnt_n ? cpos[st_n + l] : 0;
        // first pass of plane it+1 (populations kept) and, if it is output, its halo ring; all
        // loads issued before any is used.  Halo position h goes to lane (cnt + h) mod 512, the
        // lanes after the plane's own nodes (and after a second pass's, which start at lane 0),
        // so that waves with few or no own nodes take it; a wave with neither skips its loads.
        const bool own_n = l < cnt;
        const int cxn = pn & 63, cyn = pn >> 6, xn = x0 + cxn;
        const int in_ = own_n ? index_at(r, cxn, cyn) : -1;
        int si[L::Q];
        const uint32_t nbn = lds_sources<L, RX, RY, NPL>(sI, r, cxn + 2, cyn + 2, xn, a.nx, in_, si);
        const int hl = (l - cnt) & (NT - 1);
        CT fn[2][L::Q];
        double Xp0 = 0.0, Xp1 = 0.0, h0 = 0.0, h1 = 0.0;
        int hoff = -1, hi = -1;  // the halo position's offset in a moment plane, its fluid index
        bool hin = false, hout = false;
        {
            raw rn[2][L::Q], rh[2][L::Q];
            auto halo_issue = [&]() {
                if (need_next && hl < NHALO) {
                    int qx, qy;
                    halo_pos<TX, TY>(hl, qx, qy);
                    if (qy == TY) qy = rows;
                    hoff = (qy + 1) * (TX + 2) + qx + 1;
                    const int qgx = x0 + qx;
                    if (qgx >= 0 && qgx < a.nx && qy <= rows) hi = index_at(r, qx, qy);
                    hin = hi >= 0 && qgx == 0;
                    hout = hi >= 0 && qgx == a.nx - 1;
                    int hsi[L::Q];
                    lds_sources<L, RX, RY, NPL>(sI, r, qx + 2, qy + 2, qgx, a.nx, hi, hsi);
                    gather_issue<L, P>(a, hi < 0 ? 0 : hi, hsi, hin, hout, rh);
                }
            };
            auto halo_finish = [&]() {
                if (hoff >= 0) {
                    CT hf[2][L::Q];
                    gather_finish<L, P>(a, rh, hin, hout, hf, h0, h1);
                }
            };
            // a wave without a node of plane it+1 (a scalar test on its first lane) skips the pull
            if ((__builtin_amdgcn_readfirstlane(l) & ~63) < cnt) {
                gather_issue<L, P>(a, in_ < 0 ? 0 : in_, si, xn == 0, xn == a.nx - 1, rn);
                halo_issue();
                gather_finish<L, P>(a, rn, xn == 0, xn == a.nx - 1, fn, Xp0, Xp1);
                halo_finish();
            } else {
                halo_issue();
#pragma unroll
                for (int k = 0; k < L::Q; ++k) fn[0][k] = fn[1][k] = CT(0);
                halo_finish();
            }
        }
        if (in_ < 0) Xp0 = Xp1 = 0.0;
        if (hi < 0) h0 = h1 = 0.0;
        const int sn = (r + 1) & 3;
        if (own_n) {
            sX[sn][0][cyn + 1][cxn + 1] = Xp0;
            sX[sn][1][cyn + 1][cxn + 1] = Xp1;
        }
        if (hoff >= 0) {
            (&sX[sn][0][0][0])[hoff] = h0;
            (&sX[sn][1][0][0])[hoff] = h1;
        }
        // second pass of plane it+1: moments only
        for (int k = l + NT; k < cnt; k += NT) moments_to_ring(r, cpos[st + k]);
        stage_store_slot(stg, sI + (it + 5) % NPL * RY * RX);
        __syncthreads();
        // collision of plane it: the kept first pass ...
        if (ic >= 0) {
            const int cx = pc & 63, cy = pc >> 6, x = x0 + cx;
            double om0, om1;
            relax(it, cx, cy, nbc, Xc0, Xc1, x == a.nx - 1, om0, om1);
            const bool src = x >= a.src_x0;
            collide_store<L, P, false, P == P_F32>(a, ic, fc, Xc0, Xc1, om0, om1, src ? a.S0 : 0.0, src ? a.S1 : 0.0);
        }
        // ... and the second pass, pulled again
        for (int k = l + NT; k < cnt_c; k += NT) {
            const int p = cpos[st_c + k];
            const int cx = p & 63, cy = p >> 6, x = x0 + cx;
            const int i = index_at(it, cx, cy);
            int ssi[L::Q];
            const uint32_t nb = lds_sources<L, RX, RY, NPL>(sI, it, cx + 2, cy + 2, x, a.nx, i, ssi);
            CT f[2][L::Q];
            double X0, X1, om0, om1;
            gather<L, P, false>(a, i, ssi, x == 0, x == a.nx - 1, f, X0, X1);
            relax(it, cx, cy, nb, X0, X1, x == a.nx - 1, om0, om1);
            const bool src = x >= a.src_x0;
            collide_store<L, P, false, P == P_F32>(a, i, f, X0, X1, om0, om1, src ? a.S0 : 0.0, src ? a.S1 : 0.0);
        }
        ic = in_;
        pc = pn;
        nbc = nbn;
        Xc0 = Xp0;
        Xc1 = Xp1;
        cnt_c = cnt;
        st_c = st;
#pragma unroll
        for (int k = 0; k < L::Q; ++k) {
            fc[0][k] = fn[0][k];
            fc[1][k] = fn[1][k];
        }
    }
}

// ---------------------------------------------------------------------------------------------
// initial state: f*_a = w_a X (equilibrium), optionally from a [3][N] FP64 field
// ---------------------------------------------------------------------------------------------
template <class L, int P, bool NS>
__global__ void k_init(StepArgs a, const double* X, double u0, double u1)
{
    using C = Codec<P>;
    using CT = typename C::CT;
    using raw = typename C::raw;
    raw* fout = static_cast<raw*>(a.fout);
    const long long N = a.N;
    for (long long n = blockIdx.x * (long long)blockDim.x + threadIdx.x; n < N;
         n += (long long)gridDim.x * blockDim.x) {
        const int i = a.idx[n];
        if (i < 0) continue;
        // the stored state is post-collision: on the reaction layer the first collision of an
        // equilibrium start adds the source (Eq. 27) and nothing else
        const bool src = (int)(n % a.nx) >= a.src_x0;
        const double v0 = (X ? X[n] : u0) + (src ? a.S0 : 0.0);
        const double v1 = (X ? X[N + n] : u1) + (src ? a.S1 : 0.0);
        const float c0 = (float)a.c0, c1 = (float)a.c1;
        if constexpr (NS) {  // reference c = X, deviations zero
            a.xout[i] = v0;
            a.xout[a.NF + i] = v1;
#pragma unroll
            for (int k = 0; k < L::Q; ++k) {
                fout[pop_elem<L>(a, k, i)] = C::enc(0.f, 0.f);
                fout[pop_elem<L>(a, L::Q + k, i)] = C::enc(0.f, 0.f);
            }
            continue;
        }
#pragma unroll
        for (int k = 0; k < L::Q; ++k) {
            // the equilibrium w_a X in the arithmetic of the collision, so that a uniform start
            // is its fixed point
            const CT e0 = wgt<L, CT>(k) * (CT)v0, e1 = wgt<L, CT>(k) * (CT)v1;
            if constexpr (C::shifted) {
                const float wf = L::wf[k];
                fout[pop_elem<L>(a, k, i)] = C::enc(e0, wf * c0);
                fout[pop_elem<L>(a, L::Q + k, i)] = C::enc(e1, wf * c1);
            } else {
                fout[pop_elem<L>(a, k, i)] = C::enc(e0, CT(0));
                fout[pop_elem<L>(a, L::Q + k, i)] = C::enc(e1, CT(0));
            }
        }
    }
}

// moments of the stored post-collision state (collision conserves them)
template <class L, int P, bool NS>
__device__ inline void node_moments(const StepArgs& a, int i, double& X0, double& X1)
{
    using C = Codec<P>;
    using raw = typename C::raw;
    const raw* fin = static_cast<const raw*>(a.fin);
    const float c0 = (float)a.c0, c1 = (float)a.c1;
    double s0 = 0.0, s1 = 0.0;
    if constexpr (NS) {  // X = c + sum_a h_a
        s0 = a.xin[i];
        s1 = a.xin[a.NF + i];
    }
#pragma unroll
    for (int k = 0; k < L::Q; ++k) {
        if constexpr (NS) {
            s0 += (double)C::dec(fin[pop_elem<L>(a, k, i)], 0.f);
            s1 += (double)C::dec(fin[pop_elem<L>(a, L::Q + k, i)], 0.f);
        } else if constexpr (C::shifted) {
            const float wf = L::wf[k];
            s0 += (double)C::dec(fin[pop_elem<L>(a, k, i)], wf * c0);
            s1 += (double)C::dec(fin[pop_elem<L>(a, L::Q + k, i)], wf * c1);
        } else {
            s0 += (double)C::dec(fin[pop_elem<L>(a, k, i)], 0);
            s1 += (double)C::dec(fin[pop_elem<L>(a, L::Q + k, i)], 0);
        }
    }
    X0 = s0;
    X1 = s1;
}

// ---------------------------------------------------------------------------------------------
// deterministic FP64 block reduction of NV values per thread (wavefront shuffles, then LDS)
// ---------------------------------------------------------------------------------------------
template <int NV>
__device__ inline void block_reduce_store(double (&v)[NV], double* out)
{
    __shared__ double red[NV][16];
    const int lane = threadIdx.x & 63;
    const int wid = threadIdx.x >> 6;
    const int nw = (blockDim.x + 63) >> 6;
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        double s = v[i];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
        if (lane == 0) red[i][wid] = s;
    }
    __syncthreads();
    if (threadIdx.x < NV) {
        double s = 0.0;
        for (int w = 0; w < nw; ++w) s += red[threadIdx.x][w];
        out[threadIdx.x] = s;
    }
}

// residual window / inventory: per-block partial sums
//   0: sum (X - Xsnap)^2, 1: sum X^2, 2: inventory 1, 3: inventory 2, 4: non-finite count,
//   5: negative-fraction count
template <class L, int P, bool NS>
__device__ inline void residual_sums(const StepArgs& a, double* snap, int update, long long first,
                                     long long stride, double (&v)[6])
{
    const long long NF = a.NF;
    for (long long i = first; i < NF; i += stride) {
        double X0, X1;
        node_moments<L, P, NS>(a, (int)i, X0, X1);
        const double X2 = 1.0 - X0 - X1;
        if (update) {
            const double d0 = X0 - snap[i], d1 = X1 - snap[NF + i];
            v[0] += d0 * d0 + d1 * d1;
            snap[i] = X0;
            snap[NF + i] = X1;
        }
        v[1] += X0 * X0 + X1 * X1;
        v[2] += X0;
        v[3] += X1;
        const bool finite = (X0 - X0 == 0.0) && (X1 - X1 == 0.0);
        v[4] += finite ? 0.0 : 1.0;
        v[5] += (X0 < -1e-12 || X1 < -1e-12 || X2 < -1e-12) ? 1.0 : 0.0;
    }
}
template <class L, int P, bool NS>
__global__ __launch_bounds__(256) void k_residual(StepArgs a, double* snap, int update,
                                                  double* partial)
{
    double v[6] = {0, 0, 0, 0, 0, 0};
    residual_sums<L, P, NS>(a, snap, update, blockIdx.x * (long long)blockDim.x + threadIdx.x,
                            (long long)gridDim.x * blockDim.x, v);
    block_reduce_store<6>(v, partial + (long long)blockIdx.x * 8);
}
// k_residual for every instance of a batch at once: nblocks workgroups per instance, each doing
// what workgroup b of the instance's own k_residual does (the same sums in the same order)
template <class L, int P, bool NS>
__global__ __launch_bounds__(256) void k_residual_batch(const StepArgs* __restrict__ tab,
                                                        const ResidualSlot* __restrict__ slots,
                                                        int nblocks, int update)
{
    const int k = blockIdx.x / nblocks, b = blockIdx.x - k * nblocks;
    const ResidualSlot& s = slots[k];
    if (!s.active) return;  // the whole workgroup
    double v[6] = {0, 0, 0, 0, 0, 0};
    residual_sums<L, P, NS>(tab[k], s.snap, update, b * (long long)blockDim.x + threadIdx.x,
                            (long long)nblocks * blockDim.x, v);
    block_reduce_store<6>(v, s.partial + (long long)b * 8);
}

// fixed-order sum of the per-block partials (one workgroup)
__global__ __launch_bounds__(256) void k_finalize(const double* partial, int nblocks, int nv,
                                                  double* out)
{
    double v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int b = threadIdx.x; b < nblocks; b += blockDim.x)
        for (int i = 0; i < 8; ++i)
            if (i < nv) v[i] += partial[(long long)b * 8 + i];
    block_reduce_store<8>(v, out);
}

// k_finalize of each instance of a batch (workgroup k), plus its first 16 flag bytes
__global__ __launch_bounds__(256) void k_finalize_batch(const ResidualSlot* __restrict__ slots,
                                                        int nblocks, double* out)
{
    const ResidualSlot& s = slots[blockIdx.x];
    if (!s.active) return;
    double v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int b = threadIdx.x; b < nblocks; b += blockDim.x)
        for (int i = 0; i < 8; ++i)
            if (i < 6) v[i] += s.partial[(long long)b * 8 + i];
    double* o = out + (long long)blockIdx.x * 16;
    block_reduce_store<8>(v, o);
    if (threadIdx.x < 4) reinterpret_cast<unsigned*>(o + 8)[threadIdx.x] = s.flags[threadIdx.x];
}

// outlet-column means and boundary balances, over the y-z face (one thread per face node)
//   0,1: sum X_s over open outlet nodes, 2: open outlet count,
//   3,4: inflow through x = 0 during the next step, 5,6: outflow through x = nx - 1
template <class L, int P, bool NS>
__global__ __launch_bounds__(256) void k_faces(StepArgs a, double* partial)
{
    using CT = typename Codec<P>::CT;
    using C = Codec<P>;
    using raw = typename C::raw;
    const raw* fin = static_cast<const raw*>(a.fin);
    double v[7] = {0, 0, 0, 0, 0, 0, 0};
    const long long face = (long long)a.ny * a.nz;
    for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < face;
         k += (long long)gridDim.x * blockDim.x) {
        const int y = (int)(k % a.ny), z = (int)(k / a.ny);
        for (int side = 0; side < 2; ++side) {
            const int x = side ? a.nx - 1 : 0;
            const long long n = ((long long)z * a.ny + y) * a.nx + x;
            const int i = a.idx[n];
            if (i < 0) continue;
            CT f[2][L::Q];
            double X0, X1;
            pull_node<L, P, NS>(a, x, y, z, n, i, f, X0, X1);
            const float c0 = (float)a.c0, c1 = (float)a.c1;
            double cross0 = 0.0, cross1 = 0.0;  // net +x transfer across the face
#pragma unroll
            for (int q = 0; q < L::Q; ++q) {
                if (L::ex[q] == 0) continue;
                // post-stream population (NODE shift: f = w X + g)
                double p0 = (double)f[0][q], p1 = (double)f[1][q];
                if constexpr (NS) {
                    p0 += L::w[q] * X0;
                    p1 += L::w[q] * X1;
                }
                // post-collision population of this node leaving through the face
                double o0, o1;
                if constexpr (NS) {
                    o0 = L::w[q] * a.xin[i] + (double)C::dec(fin[pop_elem<L>(a, q, i)], 0.f);
                    o1 = L::w[q] * a.xin[a.NF + i] +
                         (double)C::dec(fin[pop_elem<L>(a, L::Q + q, i)], 0.f);
                } else if constexpr (C::shifted) {
                    const float wf = L::wf[q];
                    o0 = C::dec(fin[pop_elem<L>(a, q, i)], wf * c0);
                    o1 = C::dec(fin[pop_elem<L>(a, L::Q + q, i)], wf * c1);
                } else {
                    o0 = C::dec(fin[pop_elem<L>(a, q, i)], 0);
                    o1 = C::dec(fin[pop_elem<L>(a, L::Q + q, i)], 0);
                }
                if (side == 0) {
                    if (L::ex[q] == 1) { cross0 += p0; cross1 += p1; }
                    else { cross0 -= o0; cross1 -= o1; }
                } else {
                    if (L::ex[q] == 1) { cross0 += o0; cross1 += o1; }
                    else { cross0 -= p0; cross1 -= p1; }
                }
            }
            if (side == 0) {
                v[3] += cross0;
                v[4] += cross1;
            } else {
                double m0, m1;
                node_moments<L, P, NS>(a, i, m0, m1);
                // mole fractions before this step's source (the stored state is post-collision)
                const bool src = x >= a.src_x0;
                v[0] += m0 - (src ? a.S0 : 0.0);
                v[1] += m1 - (src ? a.S1 : 0.0);
                v[2] += 1.0;
                v[5] += cross0;
                v[6] += cross1;
            }
        }
    }
    block_reduce_store<7>(v, partial + (long long)blockIdx.x * 8);
}

// mole-fraction field [3][N] (solid nodes 0)
template <class L, int P, bool NS>
__global__ void k_fields(StepArgs a, double* X)
{
    const long long N = a.N;
    for (long long n = blockIdx.x * (long long)blockDim.x + threadIdx.x; n < N;
         n += (long long)gridDim.x * blockDim.x) {
        double X0 = 0.0, X1 = 0.0, X2 = 0.0;
        const int i = a.idx[n];
        if (i >= 0) {
            node_moments<L, P, NS>(a, i, X0, X1);
            if ((int)(n % a.nx) >= a.src_x0) {  // before this step's source (post-collision state)
                X0 -= a.S0;
                X1 -= a.S1;
            }
            X2 = 1.0 - X0 - X1;
        }
        X[n] = X0;
        X[N + n] = X1;
        X[2 * N + n] = X2;
    }
}

// one link plane of the decoded post-collision populations (species s, link q)
template <class L, int P, bool NS>
__global__ void k_populations(StepArgs a, int s, int q, double* out)
{
    using C = Codec<P>;
    using raw = typename C::raw;
    const raw* fin = static_cast<const raw*>(a.fin);
    const long long N = a.N;
    for (long long n = blockIdx.x * (long long)blockDim.x + threadIdx.x; n < N;
         n += (long long)gridDim.x * blockDim.x) {
        double v = 0.0;
        const int i = a.idx[n];
        if (i >= 0) {
            const float c = (float)(s ? a.c1 : a.c0);
            const raw r = fin[pop_elem<L>(a, s * L::Q + q, i)];
            if constexpr (NS) v = L::w[q] * a.xin[(long long)s * a.NF + i] + (double)C::dec(r, 0.f);
            else if constexpr (C::shifted) v = C::dec(r, L::wf[q] * c);
            else v = C::dec(r, 0);
        }
        out[n] = v;
    }
}

// The paper's initial profile along x: the flux equals the electrode flux and the generalized
// Fick law dX/dx = -[B(X)] N / C_t is integrated from the inlet composition; in lattice units
// dX/dk = -[B*(X)] Qs with Qs the superficial lattice flux.  One thread, classical RK4 with
// eight sub-steps per node spacing; writes prof[2][nx].
__global__ void k_paper_profile(StepArgs a, double Qs0, double Qs1, double* prof)
{
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    auto rhs = [&](double X0, double X1, double& d0, double& d1) {
        const double X2 = 1.0 - X0 - X1;
        const double B00 = X0 * a.iD13 + X1 * a.iD12 + X2 * a.iD13;
        const double B01 = -X0 * (a.iD12 - a.iD13);
        const double B10 = -X1 * (a.iD12 - a.iD23);
        const double B11 = X1 * a.iD23 + X0 * a.iD12 + X2 * a.iD23;
        d0 = -(B00 * Qs0 + B01 * Qs1);
        d1 = -(B10 * Qs0 + B11 * Qs1);
    };
    double X0 = a.Xin0, X1 = a.Xin1;
    const int sub = 8;
    const double h = 1.0 / sub;
    for (int x = 0; x < a.nx; ++x) {
        prof[x] = X0;
        prof[a.nx + x] = X1;
        for (int s = 0; s < sub; ++s) {
            double k10, k11, k20, k21, k30, k31, k40, k41;
            rhs(X0, X1, k10, k11);
            rhs(X0 + 0.5 * h * k10, X1 + 0.5 * h * k11, k20, k21);
            rhs(X0 + 0.5 * h * k20, X1 + 0.5 * h * k21, k30, k31);
            rhs(X0 + h * k30, X1 + h * k31, k40, k41);
            X0 += h / 6.0 * (k10 + 2.0 * k20 + 2.0 * k30 + k40);
            X1 += h / 6.0 * (k11 + 2.0 * k21 + 2.0 * k31 + k41);
        }
    }
}

__global__ void k_broadcast_profile(long long N, int nx, const double* prof, double* X)
{
    for (long long n = blockIdx.x * (long long)blockDim.x + threadIdx.x; n < N;
         n += (long long)gridDim.x * blockDim.x) {
        const int x = (int)(n % nx);
        const double v0 = prof[x], v1 = prof[nx + x];
        X[n] = v0;
        X[N + n] = v1;
        X[2 * N + n] = 1.0 - v0 - v1;
    }
}

// ---------------------------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------------------------
static inline int grid_for(long long n, int bs, int cap = 4096)
{
    long long g = (n + bs - 1) / bs;
    if (g < 1) g = 1;
    return (int)(g < cap ? g : cap);
}

template <class L, int P, bool NS>
struct Ops {
    static hipError_t init(hipStream_t st, const StepArgs& a, const double* X, double u0, double u1)
    {
        hipLaunchKernelGGL((k_init<L, P, NS>), dim3(grid_for(a.N, 256)), dim3(256), 0, st, a, X, u0, u1);
        return hipGetLastError();
    }
    static hipError_t residual(hipStream_t st, const StepArgs& a, double* snap, int update,
                               double* partial, int nblocks)
    {
        hipLaunchKernelGGL((k_residual<L, P, NS>), dim3(nblocks), dim3(256), 0, st, a, snap, update, partial);
        return hipGetLastError();
    }
    static hipError_t residual_batch(hipStream_t st, const StepArgs* tab, const ResidualSlot* slots,
                                     int count, int update, int nblocks)
    {
        hipLaunchKernelGGL((k_residual_batch<L, P, NS>), dim3(count * nblocks), dim3(256), 0, st, tab,
                           slots, nblocks, update);
        return hipGetLastError();
    }
    static hipError_t faces(hipStream_t st, const StepArgs& a, double* partial, int nblocks)
    {
        hipLaunchKernelGGL((k_faces<L, P, NS>), dim3(nblocks), dim3(256), 0, st, a, partial);
        return hipGetLastError();
    }
    static hipError_t fields(hipStream_t st, const StepArgs& a, double* X)
    {
        hipLaunchKernelGGL((k_fields<L, P, NS>), dim3(grid_for(a.N, 256)), dim3(256), 0, st, a, X);
        return hipGetLastError();
    }
    static hipError_t populations(hipStream_t st, const StepArgs& a, int s, int q, double* out)
    {
        hipLaunchKernelGGL((k_populations<L, P, NS>), dim3(grid_for(a.N, 256)), dim3(256), 0, st, a, s, q, out);
        return hipGetLastError();
    }
};

template <class L, int P, bool NS>
static hipError_t launch_step_l(hipStream_t st, const StepArgs& a, int ty, int cz, int nblocks,
                                const unsigned* coff, const unsigned short* cpos)
{
    if (ty == 12 || ty == 16) {
        if constexpr (NS || P == P_F64) {
            return hipErrorInvalidValue;
        } else {
            if (!coff || !cpos) return hipErrorInvalidValue;
            if (ty == 12 && cz == 32) hipLaunchKernelGGL((k_step3dc<L, P, 12, 32>), dim3(nblocks), dim3(512), 0, st, a, coff, cpos);
            else if (ty == 12 && cz == 64) hipLaunchKernelGGL((k_step3dc<L, P, 12, 64>), dim3(nblocks), dim3(512), 0, st, a, coff, cpos);
            else if (ty == 16 && cz == 16) hipLaunchKernelGGL((k_step3dc<L, P, 16, 16>), dim3(nblocks), dim3(512), 0, st, a, coff, cpos);
            else if (ty == 16 && cz == 32) hipLaunchKernelGGL((k_step3dc<L, P, 16, 32>), dim3(nblocks), dim3(512), 0, st, a, coff, cpos);
            else if (ty == 16 && cz == 64) hipLaunchKernelGGL((k_step3dc<L, P, 16, 64>), dim3(nblocks), dim3(512), 0, st, a, coff, cpos);
            else return hipErrorInvalidValue;
            return hipGetLastError();
        }
    }
    if (ty == 4 && cz == 16) hipLaunchKernelGGL((k_step3d<L, P, NS, 4, 16>), dim3(nblocks), dim3(256), 0, st, a);
    else if (ty == 4 && cz == 32) hipLaunchKernelGGL((k_step3d<L, P, NS, 4, 32>), dim3(nblocks), dim3(256), 0, st, a);
    else if (ty == 8 && cz == 16) hipLaunchKernelGGL((k_step3d<L, P, NS, 8, 16>), dim3(nblocks), dim3(512), 0, st, a);
    else if (ty == 8 && cz == 32) hipLaunchKernelGGL((k_step3d<L, P, NS, 8, 32>), dim3(nblocks), dim3(512), 0, st, a);
    else if (ty == 8 && cz == 64) hipLaunchKernelGGL((k_step3d<L, P, NS, 8, 64>), dim3(nblocks), dim3(512), 0, st, a);
    else if (ty == 8 && cz == 128) hipLaunchKernelGGL((k_step3d<L, P, NS, 8, 128>), dim3(nblocks), dim3(512), 0, st, a);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

template <int P, bool NS>
static hipError_t launch_step_p(hipStream_t st, const StepArgs& a, int lattice, int ty, int cz,
                                int nblocks, const unsigned* coff, const unsigned short* cpos)
{
    if (lattice == 1) return launch_step_l<D3Q19, P, NS>(st, a, ty, cz, nblocks, coff, cpos);
    if (lattice == 3) return launch_step_l<D3Q7, P, NS>(st, a, ty, cz, nblocks, coff, cpos);
    return hipErrorInvalidValue;
}

template <class L, int P, bool NS>
static hipError_t launch_step2d_p(hipStream_t st, const StepArgs* insts, const int4* tiles,
                                  const unsigned* ent, int ntiles, int ty, int rows)
{
    if (ntiles <= 0) return hipSuccess;
    if (ty == 4 && rows == 0)
        hipLaunchKernelGGL((k_step2d<L, P, NS, 4, 4>), dim3(ntiles), dim3(32 * 4), 0, st, insts, tiles, ent);
    else if (ty == 8 && rows == 0)
        hipLaunchKernelGGL((k_step2d<L, P, NS, 8, 8>), dim3(ntiles), dim3(32 * 8), 0, st, insts, tiles, ent);
    else if (ty == 16 && rows == 0)
        hipLaunchKernelGGL((k_step2d<L, P, NS, 16, 16>), dim3(ntiles), dim3(32 * 16), 0, st, insts, tiles, ent);
    else if (ty == 8 && rows == 12)
        hipLaunchKernelGGL((k_step2d<L, P, NS, 8, 12>), dim3(ntiles), dim3(32 * 8), 0, st, insts, tiles, ent);
    else if (ty == 16 && rows == 24)
        hipLaunchKernelGGL((k_step2d<L, P, NS, 16, 24>), dim3(ntiles), dim3(32 * 16), 0, st, insts, tiles, ent);
    else if (ty == 8 && rows == 9)
        hipLaunchKernelGGL((k_step2d<L, P, NS, 8, 9>), dim3(ntiles), dim3(32 * 8), 0, st, insts, tiles, ent);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

template <class L>
static hipError_t launch_step2d_l(hipStream_t st, const StepArgs* insts, const int4* tiles,
                                  const unsigned* ent, int ntiles, int prec, int node_shift, int ty,
                                  int rows)
{
    switch (prec) {
    case P_F64: return launch_step2d_p<L, P_F64, false>(st, insts, tiles, ent, ntiles, ty, rows);
    case P_F32: return node_shift ? launch_step2d_p<L, P_F32, true>(st, insts, tiles, ent, ntiles, ty, rows)
                                  : launch_step2d_p<L, P_F32, false>(st, insts, tiles, ent, ntiles, ty, rows);
    case P_F16: return node_shift ? launch_step2d_p<L, P_F16, true>(st, insts, tiles, ent, ntiles, ty, rows)
                                  : launch_step2d_p<L, P_F16, false>(st, insts, tiles, ent, ntiles, ty, rows);
    case P_BF16: return node_shift ? launch_step2d_p<L, P_BF16, true>(st, insts, tiles, ent, ntiles, ty, rows)
                                   : launch_step2d_p<L, P_BF16, false>(st, insts, tiles, ent, ntiles, ty, rows);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_step2d(hipStream_t st, const StepArgs* insts, const int4* tiles,
                         const unsigned* ent, int ntiles, int lattice, int prec, int node_shift, int ty,
                         int rows)
{
    if (lattice == 2) return launch_step2d_l<D2Q5>(st, insts, tiles, ent, ntiles, prec, node_shift, ty, rows);
    if (lattice == 0) return launch_step2d_l<D2Q9>(st, insts, tiles, ent, ntiles, prec, node_shift, ty, rows);
    return hipErrorInvalidValue;
}

int tile_options(int lattice, bool compacted, int* ty, int* cz, int cap)
{
    // 2D: (lanes / 32, 0) for fixed 64 x TY tiles, (lanes / 32, rows) for packed tiles of at
    // most `rows` rows; 3D: (TY, planes per workgroup), TY = 12 and 16 for the fluid-compacted
    // columns (global-shift storage in 32 or 16 bits only)
    static const int t2[6][2] = {{4, 0}, {8, 0}, {16, 0}, {8, 9}, {8, 12}, {16, 24}};
    static const int t3[11][2] = {{4, 16}, {4, 32}, {8, 16}, {8, 32}, {8, 64}, {8, 128},
                                  {12, 32}, {12, 64}, {16, 16}, {16, 32}, {16, 64}};
    const bool d2 = lattice == 0 || lattice == 2;  // D2Q9 and D2Q5 share the 2D launch shapes
    const int total = d2 ? 6 : (compacted ? 11 : 6);
    for (int i = 0; i < total && i < cap; ++i) {
        if (ty) ty[i] = d2 ? t2[i][0] : t3[i][0];
        if (cz) cz[i] = d2 ? t2[i][1] : t3[i][1];
    }
    return total;
}

// Workgroups of the 3D step that one CU holds at once for 64 x ty columns (the 32-plane build;
// the chunk length does not change the register or LDS footprint), 0 on error.
template <class L, int P, bool NS>
static int resident3d_l(int ty)
{
    int n = 0;
    hipError_t e = hipErrorInvalidValue;
    if (ty == 4) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_step3d<L, P, NS, 4, 32>, 256, 0);
    else if (ty == 8) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_step3d<L, P, NS, 8, 32>, 512, 0);
    if constexpr (!NS && P != P_F64) {
        if (ty == 12) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_step3dc<L, P, 12, 32>, 512, 0);
        else if (ty == 16) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_step3dc<L, P, 16, 32>, 512, 0);
    }
    return e == hipSuccess ? n : 0;
}

template <class L>
static int resident3d_p(int prec, int node_shift, int ty)
{
    switch (prec) {
    case P_F64: return resident3d_l<L, P_F64, false>(ty);
    case P_F32: return node_shift ? resident3d_l<L, P_F32, true>(ty) : resident3d_l<L, P_F32, false>(ty);
    case P_F16: return node_shift ? resident3d_l<L, P_F16, true>(ty) : resident3d_l<L, P_F16, false>(ty);
    case P_BF16: return node_shift ? resident3d_l<L, P_BF16, true>(ty) : resident3d_l<L, P_BF16, false>(ty);
    }
    return 0;
}

int step3d_resident_blocks(int lattice, int prec, int node_shift, int ty)
{
    if (lattice == 1) return resident3d_p<D3Q19>(prec, node_shift, ty);
    if (lattice == 3) return resident3d_p<D3Q7>(prec, node_shift, ty);
    return 0;
}

hipError_t launch_step(hipStream_t st, const StepArgs& a, int lattice, int prec, int node_shift,
                       int ty, int cz, int nblocks, const unsigned* coff, const unsigned short* cpos)
{
    switch (prec) {
    case P_F64: return launch_step_p<P_F64, false>(st, a, lattice, ty, cz, nblocks, coff, cpos);
    case P_F32: return node_shift ? launch_step_p<P_F32, true>(st, a, lattice, ty, cz, nblocks, coff, cpos)
                                  : launch_step_p<P_F32, false>(st, a, lattice, ty, cz, nblocks, coff, cpos);
    case P_F16: return node_shift ? launch_step_p<P_F16, true>(st, a, lattice, ty, cz, nblocks, coff, cpos)
                                  : launch_step_p<P_F16, false>(st, a, lattice, ty, cz, nblocks, coff, cpos);
    case P_BF16: return node_shift ? launch_step_p<P_BF16, true>(st, a, lattice, ty, cz, nblocks, coff, cpos)
                                   : launch_step_p<P_BF16, false>(st, a, lattice, ty, cz, nblocks, coff, cpos);
    }
    return hipErrorInvalidValue;
}

template <template <class, int, bool> class Fn, class... Args>
static hipError_t dispatch(int lattice, int prec, int ns, Args&&... args)
{
#define LBMMS_CASES(LAT)                                                                   \
    switch (prec) {                                                                        \
    case P_F64: return Fn<LAT, P_F64, false>::run(args...);                                \
    case P_F32: return ns ? Fn<LAT, P_F32, true>::run(args...) : Fn<LAT, P_F32, false>::run(args...); \
    case P_F16: return ns ? Fn<LAT, P_F16, true>::run(args...) : Fn<LAT, P_F16, false>::run(args...); \
    case P_BF16: return ns ? Fn<LAT, P_BF16, true>::run(args...) : Fn<LAT, P_BF16, false>::run(args...); \
    }
    if (lattice == 0) { LBMMS_CASES(D2Q9) }
    else if (lattice == 2) { LBMMS_CASES(D2Q5) }
    else if (lattice == 3) { LBMMS_CASES(D3Q7) }
    else { LBMMS_CASES(D3Q19) }
#undef LBMMS_CASES
    return hipErrorInvalidValue;
}

template <class L, int P, bool NS> struct RunInit {
    static hipError_t run(hipStream_t st, const StepArgs& a, const double* X, double u0, double u1)
    { return Ops<L, P, NS>::init(st, a, X, u0, u1); }
};
template <class L, int P, bool NS> struct RunResidual {
    static hipError_t run(hipStream_t st, const StepArgs& a, double* snap, int upd, double* part, int nb)
    { return Ops<L, P, NS>::residual(st, a, snap, upd, part, nb); }
};
template <class L, int P, bool NS> struct RunResidualBatch {
    static hipError_t run(hipStream_t st, const StepArgs* tab, const ResidualSlot* slots, int count,
                          int upd, int nb)
    { return Ops<L, P, NS>::residual_batch(st, tab, slots, count, upd, nb); }
};
template <class L, int P, bool NS> struct RunFaces {
    static hipError_t run(hipStream_t st, const StepArgs& a, double* part, int nb)
    { return Ops<L, P, NS>::faces(st, a, part, nb); }
};
template <class L, int P, bool NS> struct RunFields {
    static hipError_t run(hipStream_t st, const StepArgs& a, double* X)
    { return Ops<L, P, NS>::fields(st, a, X); }
};
template <class L, int P, bool NS> struct RunPops {
    static hipError_t run(hipStream_t st, const StepArgs& a, int s, int q, double* out)
    { return Ops<L, P, NS>::populations(st, a, s, q, out); }
};

hipError_t launch_init(hipStream_t st, const StepArgs& a, int lattice, int prec, int ns,
                       const double* X, double u0, double u1)
{
    return dispatch<RunInit>(lattice, prec, ns, st, a, X, u0, u1);
}

hipError_t launch_residual(hipStream_t st, const StepArgs& a, int lattice, int prec, int ns,
                           double* snap, int update, double* partial, int nblocks, double* out)
{
    hipError_t e = dispatch<RunResidual>(lattice, prec, ns, st, a, snap, update, partial, nblocks);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(256), 0, st, partial, nblocks, 6, out);
    return hipGetLastError();
}

hipError_t launch_residual_batch(hipStream_t st, const StepArgs* tab, const ResidualSlot* slots,
                                 int count, int lattice, int prec, int ns, int update, int nblocks,
                                 double* out)
{
    hipError_t e = dispatch<RunResidualBatch>(lattice, prec, ns, st, tab, slots, count, update, nblocks);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_finalize_batch, dim3(count), dim3(256), 0, st, slots, nblocks, out);
    return hipGetLastError();
}

hipError_t launch_faces(hipStream_t st, const StepArgs& a, int lattice, int prec, int ns,
                        double* partial, int nblocks, double* out)
{
    hipError_t e = dispatch<RunFaces>(lattice, prec, ns, st, a, partial, nblocks);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(256), 0, st, partial, nblocks, 7, out);
    return hipGetLastError();
}

hipError_t launch_fields(hipStream_t st, const StepArgs& a, int lattice, int prec, int ns, double* X)
{
    return dispatch<RunFields>(lattice, prec, ns, st, a, X);
}

hipError_t launch_populations(hipStream_t st, const StepArgs& a, int lattice, int prec, int ns,
                              int s, int q, double* out)
{
    return dispatch<RunPops>(lattice, prec, ns, st, a, s, q, out);
}

hipError_t launch_paper_profile(hipStream_t st, const StepArgs& a, double Qs0, double Qs1,
                                double* prof, double* X)
{
    hipLaunchKernelGGL(k_paper_profile, dim3(1), dim3(64), 0, st, a, Qs0, Qs1, prof);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_broadcast_profile, dim3(grid_for(a.N, 256)), dim3(256), 0, st, a.N, a.nx, prof, X);
    return hipGetLastError();
}

}  // namespace lbmms
