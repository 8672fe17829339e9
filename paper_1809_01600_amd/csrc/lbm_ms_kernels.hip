// HIP kernels (gfx950) of the LBM / Maxwell-Stefan time step and its reductions.
//
// Step kernels are pull-scheme and fused: each fluid node pulls its post-collision populations
// from the neighbours (bounce-back and the x-boundary rules applied on the way), forms the
// moments, takes the mole-fraction gradients from an LDS tile that also holds a one-node halo
// (recomputed from the halo nodes' own pulls), solves the Maxwell-Stefan system in FP64 for the
// relaxation times, collides and stores to the other buffer.  Populations are structure of
// arrays [species][link][node] with x fastest, so a wavefront's loads and stores are coalesced
// along x.
#include <hip/hip_runtime.h>

#include "lbm_ms_device.hpp"
#include "lbm_ms_kernels.hpp"

namespace lbmms {

// ---------------------------------------------------------------------------------------------
// 2D (D2Q9): one workgroup = 64 x TY output tile + one-node halo ring, all pulls in flight at once
// ---------------------------------------------------------------------------------------------
template <int P, bool NS, int TY>
__global__ __launch_bounds__(64 * TY) void k_step2d(StepArgs a)
{
    using L = D2Q9;
    using CT = typename Codec<P>::CT;
    constexpr int TX = 64;
    __shared__ double sX[2][TY + 2][TX + 2];

    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int x0 = (tile % a.tiles_x) * TX;
    const int y0 = (tile / a.tiles_x) * TY;
    const int lx = threadIdx.x & (TX - 1);
    const int ly = threadIdx.x / TX;
    const int x = x0 + lx;
    const int yr = y0 + ly;
    const int y = yr % a.ny;  // rows past the end hold the periodic image
    const bool own = (x < a.nx) && (yr < a.ny);
    const long long n = (long long)y * a.nx + x;
    const uint32_t d = (x < a.nx) ? a.desc[n] : 0u;

    CT f[2][L::Q];
    double X0 = 0.0, X1 = 0.0;
    if (d & FLUID) pull_node<L, P, NS>(a, x, y, 0, n, d, f, X0, X1);
    sX[0][ly + 1][lx + 1] = X0;
    sX[1][ly + 1][lx + 1] = X1;

    // halo ring: row below, row above, column left, column right
    const int t = threadIdx.x;
    if (t < 2 * TX + 2 * TY) {
        int hx, hyr, sx, sy;
        if (t < TX) { hx = x0 + t; hyr = y0 - 1; sx = t + 1; sy = 0; }
        else if (t < 2 * TX) { hx = x0 + t - TX; hyr = y0 + TY; sx = t - TX + 1; sy = TY + 1; }
        else if (t < 2 * TX + TY) { hx = x0 - 1; hyr = y0 + t - 2 * TX; sx = 0; sy = t - 2 * TX + 1; }
        else { hx = x0 + TX; hyr = y0 + t - 2 * TX - TY; sx = TX + 1; sy = t - 2 * TX - TY + 1; }
        const int hy = ((hyr % a.ny) + a.ny) % a.ny;
        double h0 = 0.0, h1 = 0.0;
        if (hx >= 0 && hx < a.nx) {
            const long long hn = (long long)hy * a.nx + hx;
            const uint32_t hd = a.desc[hn];
            if (hd & FLUID) {
                CT hf[2][L::Q];
                pull_node<L, P, NS>(a, hx, hy, 0, hn, hd, hf, h0, h1);
            }
        }
        sX[0][sy][sx] = h0;
        sX[1][sy][sx] = h1;
    }
    __syncthreads();

    if (own && (d & FLUID)) {
        double g0[3], g1[3];
        const int cx = lx + 1, cy = ly + 1;
        const bool xp = d & NB_XP, xm = d & NB_XM, yp = d & NB_YP, ym = d & NB_YM;
        g0[0] = grad1(xp, xm, sX[0][cy][cx + 1], X0, sX[0][cy][cx - 1]);
        g1[0] = grad1(xp, xm, sX[1][cy][cx + 1], X1, sX[1][cy][cx - 1]);
        g0[1] = grad1(yp, ym, sX[0][cy + 1][cx], X0, sX[0][cy - 1][cx]);
        g1[1] = grad1(yp, ym, sX[1][cy + 1][cx], X1, sX[1][cy - 1][cx]);
        g0[2] = g1[2] = 0.0;
        double om0, om1;
        bool hit;
        ms_relax<2>(a, X0, X1, g0, g1, (d & OUTLET) != 0, om0, om1, hit);
        if (hit) a.flags[0] = 1u;
        collide_store<L, P, NS>(a, n, f, X0, X1, om0, om1);
    }
}

// ---------------------------------------------------------------------------------------------
// 3D (D3Q19): one workgroup = 64 x TY column tile marching through CZ planes; x/y gradients
// from a 3-slot LDS ring of planes (tile + halo ring), z gradients from the column's own
// rolling registers.  One barrier per plane.
// ---------------------------------------------------------------------------------------------
template <int P, bool NS, int TY>
__device__ inline void plane_halo(const StepArgs& a, int x0, int y0, int z, double (*sX)[TY + 2][66])
{
    using L = D3Q19;
    using CT = typename Codec<P>::CT;
    constexpr int TX = 64;
    const int t = threadIdx.x;
    if (t < 2 * TX + 2 * TY) {
        int hx, hyr, sx, sy;
        if (t < TX) { hx = x0 + t; hyr = y0 - 1; sx = t + 1; sy = 0; }
        else if (t < 2 * TX) { hx = x0 + t - TX; hyr = y0 + TY; sx = t - TX + 1; sy = TY + 1; }
        else if (t < 2 * TX + TY) { hx = x0 - 1; hyr = y0 + t - 2 * TX; sx = 0; sy = t - 2 * TX + 1; }
        else { hx = x0 + TX; hyr = y0 + t - 2 * TX - TY; sx = TX + 1; sy = t - 2 * TX - TY + 1; }
        const int hy = ((hyr % a.ny) + a.ny) % a.ny;
        double h0 = 0.0, h1 = 0.0;
        if (hx >= 0 && hx < a.nx) {
            const long long hn = ((long long)z * a.ny + hy) * a.nx + hx;
            const uint32_t hd = a.desc[hn];
            if (hd & FLUID) {
                CT hf[2][L::Q];
                pull_node<L, P, NS>(a, hx, hy, z, hn, hd, hf, h0, h1);
            }
        }
        sX[0][sy][sx] = h0;
        sX[1][sy][sx] = h1;
    }
}

template <int P, bool NS, int TY, int CZ>
__global__ __launch_bounds__(64 * TY) void k_step3d(StepArgs a)
{
    using L = D3Q19;
    using CT = typename Codec<P>::CT;
    constexpr int TX = 64;
    __shared__ double sX[3][2][TY + 2][TX + 2];

    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int bx = tile % a.tiles_x;
    const int rest = tile / a.tiles_x;
    const int by = rest % a.tiles_y;
    const int bz = rest / a.tiles_y;
    const int x0 = bx * TX, y0 = by * TY, z0 = bz * CZ;
    const int lx = threadIdx.x & (TX - 1);
    const int ly = threadIdx.x / TX;
    const int x = x0 + lx;
    const int yr = y0 + ly;
    const int y = yr % a.ny;
    const bool own = (x < a.nx) && (yr < a.ny);
    const long long plane = (long long)a.nx * a.ny;
    const long long col = (long long)y * a.nx + x;

    // plane z0 - 1 (periodic): moments only, for the z gradient of plane z0
    double Xm0 = 0.0, Xm1 = 0.0;
    {
        const int zm = (z0 == 0) ? a.nz - 1 : z0 - 1;
        const long long nm = zm * plane + col;
        const uint32_t dm = (x < a.nx) ? a.desc[nm] : 0u;
        if (dm & FLUID) {
            CT tf[2][L::Q];
            pull_node<L, P, NS>(a, x, y, zm, nm, dm, tf, Xm0, Xm1);
        }
    }
    // plane z0: populations kept for the collision, moments into LDS slot 0
    CT fc[2][L::Q];
    double Xc0 = 0.0, Xc1 = 0.0;
    uint32_t dc = (x < a.nx) ? a.desc[z0 * plane + col] : 0u;
    if (dc & FLUID) pull_node<L, P, NS>(a, x, y, z0, z0 * plane + col, dc, fc, Xc0, Xc1);
    sX[0][0][ly + 1][lx + 1] = Xc0;
    sX[0][1][ly + 1][lx + 1] = Xc1;
    plane_halo<P, NS, TY>(a, x0, y0, z0, sX[0]);

    for (int i = 0; i < CZ; ++i) {
        const int zi = z0 + i;
        if (zi >= a.nz) break;  // uniform across the workgroup
        const int zp = (zi + 1 == a.nz) ? 0 : zi + 1;
        const long long np = zp * plane + col;
        const uint32_t dn = (x < a.nx) ? a.desc[np] : 0u;
        CT fn[2][L::Q];
        double Xp0 = 0.0, Xp1 = 0.0;
        if (dn & FLUID) pull_node<L, P, NS>(a, x, y, zp, np, dn, fn, Xp0, Xp1);
        const bool need_next = (i + 1 < CZ) && (zi + 1 < a.nz);
        if (need_next) {
            const int s = (i + 1) % 3;
            sX[s][0][ly + 1][lx + 1] = Xp0;
            sX[s][1][ly + 1][lx + 1] = Xp1;
            plane_halo<P, NS, TY>(a, x0, y0, zp, sX[s]);
        }
        __syncthreads();
        if (own && (dc & FLUID)) {
            const int s = i % 3;
            const int cx = lx + 1, cy = ly + 1;
            double g0[3], g1[3];
            const bool xp = dc & NB_XP, xm = dc & NB_XM, yp = dc & NB_YP, ym = dc & NB_YM;
            const bool zpf = dc & NB_ZP, zmf = dc & NB_ZM;
            g0[0] = grad1(xp, xm, sX[s][0][cy][cx + 1], Xc0, sX[s][0][cy][cx - 1]);
            g1[0] = grad1(xp, xm, sX[s][1][cy][cx + 1], Xc1, sX[s][1][cy][cx - 1]);
            g0[1] = grad1(yp, ym, sX[s][0][cy + 1][cx], Xc0, sX[s][0][cy - 1][cx]);
            g1[1] = grad1(yp, ym, sX[s][1][cy + 1][cx], Xc1, sX[s][1][cy - 1][cx]);
            g0[2] = grad1(zpf, zmf, Xp0, Xc0, Xm0);
            g1[2] = grad1(zpf, zmf, Xp1, Xc1, Xm1);
            double om0, om1;
            bool hit;
            ms_relax<3>(a, Xc0, Xc1, g0, g1, (dc & OUTLET) != 0, om0, om1, hit);
            if (hit) a.flags[0] = 1u;
            collide_store<L, P, NS>(a, (long long)zi * plane + col, fc, Xc0, Xc1, om0, om1);
        }
        Xm0 = Xc0; Xm1 = Xc1;
        Xc0 = Xp0; Xc1 = Xp1;
        dc = dn;
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
        const bool fl = a.desc[n] & FLUID;
        const double v0 = fl ? (X ? X[n] : u0) : 0.0;
        const double v1 = fl ? (X ? X[N + n] : u1) : 0.0;
        float c0 = (float)a.c0, c1 = (float)a.c1;
        if constexpr (NS) {
            c0 = (float)v0;
            c1 = (float)v1;
            a.xout[n] = c0;
            a.xout[N + n] = c1;
        }
#pragma unroll
        for (int k = 0; k < L::Q; ++k) {
            const CT e0 = (CT)(L::w[k] * v0), e1 = (CT)(L::w[k] * v1);
            if constexpr (C::shifted) {
                const float wf = (float)L::w[k];
                fout[(long long)k * N + n] = fl ? C::enc(e0, wf * c0) : (raw)0.0f;
                fout[(long long)(L::Q + k) * N + n] = fl ? C::enc(e1, wf * c1) : (raw)0.0f;
            } else {
                fout[(long long)k * N + n] = C::enc(e0, CT(0));
                fout[(long long)(L::Q + k) * N + n] = C::enc(e1, CT(0));
            }
        }
    }
}

// moments of the stored post-collision state (collision conserves them)
template <class L, int P, bool NS>
__device__ inline void node_moments(const StepArgs& a, long long n, double& X0, double& X1)
{
    using C = Codec<P>;
    using raw = typename C::raw;
    const raw* fin = static_cast<const raw*>(a.fin);
    const long long N = a.N;
    float c0 = (float)a.c0, c1 = (float)a.c1;
    if constexpr (NS) {
        c0 = a.xin[n];
        c1 = a.xin[N + n];
    }
    double s0 = 0.0, s1 = 0.0;
#pragma unroll
    for (int k = 0; k < L::Q; ++k) {
        if constexpr (C::shifted) {
            const float wf = (float)L::w[k];
            s0 += (double)C::dec(fin[(long long)k * N + n], wf * c0);
            s1 += (double)C::dec(fin[(long long)(L::Q + k) * N + n], wf * c1);
        } else {
            s0 += (double)C::dec(fin[(long long)k * N + n], 0);
            s1 += (double)C::dec(fin[(long long)(L::Q + k) * N + n], 0);
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
__global__ __launch_bounds__(256) void k_residual(StepArgs a, double* snap, int update,
                                                  double* partial)
{
    double v[6] = {0, 0, 0, 0, 0, 0};
    const long long N = a.N;
    for (long long n = blockIdx.x * (long long)blockDim.x + threadIdx.x; n < N;
         n += (long long)gridDim.x * blockDim.x) {
        if (!(a.desc[n] & FLUID)) continue;
        double X0, X1;
        node_moments<L, P, NS>(a, n, X0, X1);
        const double X2 = 1.0 - X0 - X1;
        if (update) {
            const double d0 = X0 - snap[n], d1 = X1 - snap[N + n];
            v[0] += d0 * d0 + d1 * d1;
            snap[n] = X0;
            snap[N + n] = X1;
        }
        v[1] += X0 * X0 + X1 * X1;
        v[2] += X0;
        v[3] += X1;
        const bool finite = (X0 - X0 == 0.0) && (X1 - X1 == 0.0);
        v[4] += finite ? 0.0 : 1.0;
        v[5] += (X0 < -1e-12 || X1 < -1e-12 || X2 < -1e-12) ? 1.0 : 0.0;
    }
    block_reduce_store<6>(v, partial + (long long)blockIdx.x * 8);
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
    const long long N = a.N;
    for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < face;
         k += (long long)gridDim.x * blockDim.x) {
        const int y = (int)(k % a.ny), z = (int)(k / a.ny);
        for (int side = 0; side < 2; ++side) {
            const int x = side ? a.nx - 1 : 0;
            const long long n = ((long long)z * a.ny + y) * a.nx + x;
            const uint32_t d = a.desc[n];
            if (!(d & FLUID)) continue;
            CT f[2][L::Q];
            double X0, X1;
            pull_node<L, P, NS>(a, x, y, z, n, d, f, X0, X1);
            float c0 = (float)a.c0, c1 = (float)a.c1;
            if constexpr (NS) {
                c0 = a.xin[n];
                c1 = a.xin[N + n];
            }
            double cross0 = 0.0, cross1 = 0.0;  // net +x transfer across the face
#pragma unroll
            for (int q = 0; q < L::Q; ++q) {
                if (L::ex[q] == 0) continue;
                // post-collision population of this node leaving through the face
                double o0, o1;
                if constexpr (C::shifted) {
                    const float wf = (float)L::w[q];
                    o0 = C::dec(fin[(long long)q * N + n], wf * c0);
                    o1 = C::dec(fin[(long long)(L::Q + q) * N + n], wf * c1);
                } else {
                    o0 = C::dec(fin[(long long)q * N + n], 0);
                    o1 = C::dec(fin[(long long)(L::Q + q) * N + n], 0);
                }
                if (side == 0) {
                    if (L::ex[q] == 1) { cross0 += (double)f[0][q]; cross1 += (double)f[1][q]; }
                    else { cross0 -= o0; cross1 -= o1; }
                } else {
                    if (L::ex[q] == 1) { cross0 += o0; cross1 += o1; }
                    else { cross0 -= (double)f[0][q]; cross1 -= (double)f[1][q]; }
                }
            }
            if (side == 0) {
                v[3] += cross0;
                v[4] += cross1;
            } else {
                double m0, m1;
                node_moments<L, P, NS>(a, n, m0, m1);
                v[0] += m0;
                v[1] += m1;
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
        if (a.desc[n] & FLUID) {
            node_moments<L, P, NS>(a, n, X0, X1);
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
        if (a.desc[n] & FLUID) {
            float c = (float)(s ? a.c1 : a.c0);
            if constexpr (NS) c = a.xin[(long long)s * N + n];
            const raw r = fin[((long long)s * L::Q + q) * N + n];
            if constexpr (C::shifted) v = C::dec(r, (float)L::w[q] * c);
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

template <int P, bool NS>
static hipError_t launch_step_p(hipStream_t st, const StepArgs& a, int lattice, int ty, int cz,
                                int nblocks)
{
    if (lattice == 0) {
        switch (ty) {
        case 4: hipLaunchKernelGGL((k_step2d<P, NS, 4>), dim3(nblocks), dim3(64 * 4), 0, st, a); break;
        case 8: hipLaunchKernelGGL((k_step2d<P, NS, 8>), dim3(nblocks), dim3(64 * 8), 0, st, a); break;
        case 16: hipLaunchKernelGGL((k_step2d<P, NS, 16>), dim3(nblocks), dim3(64 * 16), 0, st, a); break;
        default: return hipErrorInvalidValue;
        }
    } else {
        if (ty == 4 && cz == 16) hipLaunchKernelGGL((k_step3d<P, NS, 4, 16>), dim3(nblocks), dim3(256), 0, st, a);
        else if (ty == 4 && cz == 32) hipLaunchKernelGGL((k_step3d<P, NS, 4, 32>), dim3(nblocks), dim3(256), 0, st, a);
        else if (ty == 8 && cz == 16) hipLaunchKernelGGL((k_step3d<P, NS, 8, 16>), dim3(nblocks), dim3(512), 0, st, a);
        else if (ty == 8 && cz == 32) hipLaunchKernelGGL((k_step3d<P, NS, 8, 32>), dim3(nblocks), dim3(512), 0, st, a);
        else return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

int tile_options(int lattice, int* ty, int* cz, int cap)
{
    static const int t2[3] = {4, 8, 16};
    static const int t3[4][2] = {{4, 16}, {4, 32}, {8, 16}, {8, 32}};
    const int total = (lattice == 0) ? 3 : 4;
    for (int i = 0; i < total && i < cap; ++i) {
        if (ty) ty[i] = (lattice == 0) ? t2[i] : t3[i][0];
        if (cz) cz[i] = (lattice == 0) ? 0 : t3[i][1];
    }
    return total;
}

hipError_t launch_step(hipStream_t st, const StepArgs& a, int lattice, int prec, int node_shift,
                       int ty, int cz, int nblocks)
{
    switch (prec) {
    case P_F64: return launch_step_p<P_F64, false>(st, a, lattice, ty, cz, nblocks);
    case P_F32: return launch_step_p<P_F32, false>(st, a, lattice, ty, cz, nblocks);
    case P_F16: return node_shift ? launch_step_p<P_F16, true>(st, a, lattice, ty, cz, nblocks)
                                  : launch_step_p<P_F16, false>(st, a, lattice, ty, cz, nblocks);
    case P_BF16: return node_shift ? launch_step_p<P_BF16, true>(st, a, lattice, ty, cz, nblocks)
                                   : launch_step_p<P_BF16, false>(st, a, lattice, ty, cz, nblocks);
    }
    return hipErrorInvalidValue;
}

template <template <class, int, bool> class Fn, class... Args>
static hipError_t dispatch(int lattice, int prec, int ns, Args&&... args)
{
#define LBMMS_CASES(LAT)                                                                   \
    switch (prec) {                                                                        \
    case P_F64: return Fn<LAT, P_F64, false>::run(args...);                                \
    case P_F32: return Fn<LAT, P_F32, false>::run(args...);                                \
    case P_F16: return ns ? Fn<LAT, P_F16, true>::run(args...) : Fn<LAT, P_F16, false>::run(args...); \
    case P_BF16: return ns ? Fn<LAT, P_BF16, true>::run(args...) : Fn<LAT, P_BF16, false>::run(args...); \
    }
    if (lattice == 0) { LBMMS_CASES(D2Q9) }
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
