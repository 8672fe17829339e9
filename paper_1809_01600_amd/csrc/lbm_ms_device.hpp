// Device-side building blocks of one time step of the LBM / Maxwell-Stefan method
// (arXiv 1809.01600): velocity sets, population storage codecs, the pull with its boundary
// rules, and the FP64 Maxwell-Stefan relaxation-time solve.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbmms {

// ---------------------------------------------------------------------------------------------
// node descriptor bits (one uint32 per node, built on the host from the cleaned mask)
// ---------------------------------------------------------------------------------------------
constexpr uint32_t BB_MASK = (1u << 19) - 1;  // bit a: the pull source of link a is solid
constexpr uint32_t NB_XM = 1u << 19;          // neighbour x-1 exists and is fluid
constexpr uint32_t NB_XP = 1u << 20;          // neighbour x+1 exists and is fluid
constexpr uint32_t NB_YM = 1u << 21;          // neighbour y-1 (periodic) is fluid
constexpr uint32_t NB_YP = 1u << 22;
constexpr uint32_t NB_ZM = 1u << 23;
constexpr uint32_t NB_ZP = 1u << 24;
constexpr uint32_t FLUID = 1u << 28;
constexpr uint32_t INLET = 1u << 29;          // x == 0
constexpr uint32_t OUTLET = 1u << 30;         // x == nx - 1

// ---------------------------------------------------------------------------------------------
// velocity sets
// ---------------------------------------------------------------------------------------------
// D2Q9 in the order of Eq. 2 (rest, the four axis links counter-clockwise from +x, then the
// diagonals from (1,1)), weights of Eq. 9.
struct D2Q9 {
    static constexpr int Q = 9;
    static constexpr int DIMS = 2;
    static constexpr int ex[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
    static constexpr int ey[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
    static constexpr int ez[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    static constexpr int opp[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
    static constexpr double w[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9,
                                    1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
};

// D3Q19 with opposite links adjacent: rest, +-x, +-y, +-z, then the twelve edge vectors.
struct D3Q19 {
    static constexpr int Q = 19;
    static constexpr int DIMS = 3;
    static constexpr int ex[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
    static constexpr int ey[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
    static constexpr int ez[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
    static constexpr int opp[19] = {0, 2, 1, 4, 3, 6, 5, 8, 7, 10, 9, 12, 11, 14, 13, 16, 15, 18, 17};
    static constexpr double w[19] = {1.0 / 3,  1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18,
                                     1.0 / 18, 1.0 / 18, 1.0 / 36, 1.0 / 36, 1.0 / 36,
                                     1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36,
                                     1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
};

// sum of the weights of the links with e_x = +1 (1/6 for both sets)
constexpr double W_OUT = 1.0 / 6.0;

// ---------------------------------------------------------------------------------------------
// population storage
// ---------------------------------------------------------------------------------------------
enum Prec { P_F64 = 0, P_F32 = 1, P_F16 = 2, P_BF16 = 3 };

template <int P> struct Codec;
template <> struct Codec<P_F64> {
    using raw = double;
    using CT = double;
    static constexpr bool shifted = false;
    __device__ static inline CT dec(raw r, CT) { return r; }
    __device__ static inline raw enc(CT v, CT) { return v; }
};
template <> struct Codec<P_F32> {
    using raw = float;
    using CT = float;
    static constexpr bool shifted = false;
    __device__ static inline CT dec(raw r, CT) { return r; }
    __device__ static inline raw enc(CT v, CT) { return v; }
};
// 16-bit storage of the shifted population h = f - s (s = w_a c)
template <> struct Codec<P_F16> {
    using raw = _Float16;
    using CT = float;
    static constexpr bool shifted = true;
    __device__ static inline CT dec(raw r, CT s) { return (float)r + s; }
    __device__ static inline raw enc(CT v, CT s) { return (_Float16)(v - s); }
};
template <> struct Codec<P_BF16> {
    using raw = __bf16;
    using CT = float;
    static constexpr bool shifted = true;
    __device__ static inline CT dec(raw r, CT s) { return (float)r + s; }
    __device__ static inline raw enc(CT v, CT s) { return (__bf16)(v - s); }
};

// ---------------------------------------------------------------------------------------------
// per-launch arguments
// ---------------------------------------------------------------------------------------------
struct StepArgs {
    const void* fin;          // post-collision populations of step t   [2][Q][N]
    void* fout;               // post-collision populations of step t+1 [2][Q][N]
    const float* xin;         // node shift field of step t   [2][N] (NODE shift only)
    float* xout;              // node shift field of step t+1 [2][N]
    const uint32_t* desc;     // node descriptors [N]
    unsigned* flags;          // [0]: relaxation time clamped
    long long N;
    int nx, ny, nz;
    int tiles_x, tiles_y, chunks_z;
    double iD12, iD13, iD23;  // 1 / D*_ij (lattice units)
    double Xin0, Xin1;        // inlet mole fractions (Dirichlet rule, Eq. 36)
    double Q0, Q1;            // lattice outflow per open outlet node (Eq. 39 scaled)
    double eps0, eps1;        // eps * |nu_1|, eps * |nu_2| (flux-norm regularizer)
    double sgn12;             // sigma_1 * sigma_2, sigma_i = -sgn(nu_i) (Eq. 24 sign rule)
    double rst21, rst12;      // stoichiometric ratios |nu_2|/|nu_1|, |nu_1|/|nu_2|
    double c0, c1;            // global shift composition (16-bit GLOBAL storage)
    double tau_min, tau_max;
    int ms_mode;              // 0 local flux norms, 1 stoichiometric ratio
    int inlet_wall;           // 1: x = 0 face is a bounce-back wall
};

// Map the hardware block index to a tile so that each of the 8 XCDs (blocks are dealt to XCDs
// round-robin) works on one contiguous band of tiles and shares halo rows through its own L2.
__device__ inline int xcd_tile(int b, int nb)
{
    const int per = nb >> 3, rem = nb & 7;
    const int xcd = b & 7, k = b >> 3;
    return (xcd < rem ? xcd * (per + 1) : rem * (per + 1) + (xcd - rem) * per) + k;
}

// ---------------------------------------------------------------------------------------------
// pull-stream of one fluid node with bounce-back and the x-boundary rules
// ---------------------------------------------------------------------------------------------
// Returns the post-stream populations f[s][a] of node n = (x, y, z) and their moments X0, X1
// (FP64 sums).  Source of link a is r - e_a.  Links whose source is solid bounce back
// (f_a(r) = f*_abar(r)); at the outlet column the links from x = nx take the exact-flux rule
// f_a = f*_abar - (w_abar / W_out) Q_s; at the inlet column the links from x = -1 take
// f_a = (w_a + w_abar) X_in - f_abar (Eq. 36) with f_abar the value just pulled, or bounce back
// when the inlet is a wall.
template <class L, int P, bool NS>
__device__ inline void pull_node(const StepArgs& a, int x, int y, int z, long long n, uint32_t d,
                                 typename Codec<P>::CT (&f)[2][L::Q], double& X0, double& X1)
{
    using C = Codec<P>;
    using CT = typename C::CT;
    using raw = typename C::raw;
    const raw* __restrict__ fin = static_cast<const raw*>(a.fin);
    const long long N = a.N;
    const long long nx = a.nx;
    const long long plane = nx * a.ny;
    // offsets of the y / z neighbours, periodic
    const long long oym = (y > 0) ? -nx : (long long)(a.ny - 1) * nx;
    const long long oyp = (y < a.ny - 1) ? nx : -(long long)(a.ny - 1) * nx;
    const long long ozm = (z > 0) ? -plane : (long long)(a.nz - 1) * plane;
    const long long ozp = (z < a.nz - 1) ? plane : -(long long)(a.nz - 1) * plane;
    const bool inlet = (d & INLET) != 0;
    const bool outlet = (d & OUTLET) != 0;

    float sh_own0 = 0.f, sh_own1 = 0.f;
    if constexpr (NS) {
        sh_own0 = a.xin[n];
        sh_own1 = a.xin[N + n];
    }
    const float cg0 = (float)a.c0, cg1 = (float)a.c1;

#pragma unroll
    for (int k = 0; k < L::Q; ++k) {
        const int ex = L::ex[k], ey = L::ey[k], ez = L::ez[k];
        const bool from_out = (ex == -1) && outlet;  // source at x = nx
        const bool from_in = (ex == 1) && inlet;     // source at x = -1
        const bool reflect = ((d >> k) & 1u) || from_out || (from_in && a.inlet_wall);
        long long src = n - ex;
        if (ey == 1) src += oym;
        if (ey == -1) src += oyp;
        if (ez == 1) src += ozm;
        if (ez == -1) src += ozp;
        if (from_in) src = n;  // placeholder, replaced below (keeps the address valid)
        const int kk = reflect ? L::opp[k] : k;
        const long long m = reflect ? n : src;
        const raw r0 = fin[(long long)kk * N + m];
        const raw r1 = fin[(long long)(L::Q + kk) * N + m];
        if constexpr (C::shifted) {
            const float wk = (float)L::w[kk];
            float s0, s1;
            if constexpr (NS) {
                s0 = wk * (reflect ? sh_own0 : a.xin[m]);
                s1 = wk * (reflect ? sh_own1 : a.xin[N + m]);
            } else {
                s0 = wk * cg0;
                s1 = wk * cg1;
            }
            f[0][k] = C::dec(r0, s0);
            f[1][k] = C::dec(r1, s1);
        } else {
            f[0][k] = C::dec(r0, CT(0));
            f[1][k] = C::dec(r1, CT(0));
        }
        if (from_out) {
            const CT frac = (CT)(L::w[L::opp[k]] / W_OUT);
            f[0][k] -= frac * (CT)a.Q0;
            f[1][k] -= frac * (CT)a.Q1;
        }
    }
    if (inlet && !a.inlet_wall) {
#pragma unroll
        for (int k = 0; k < L::Q; ++k) {
            if (L::ex[k] == 1) {
                const CT ww = (CT)(L::w[k] + L::w[L::opp[k]]);
                f[0][k] = ww * (CT)a.Xin0 - f[0][L::opp[k]];
                f[1][k] = ww * (CT)a.Xin1 - f[1][L::opp[k]];
            }
        }
    }
    double s0 = 0.0, s1 = 0.0;
#pragma unroll
    for (int k = 0; k < L::Q; ++k) {
        s0 += (double)f[0][k];
        s1 += (double)f[1][k];
    }
    X0 = s0;
    X1 = s1;
}

// ---------------------------------------------------------------------------------------------
// Maxwell-Stefan flux solve and relaxation times (FP64)
// ---------------------------------------------------------------------------------------------
// g0/g1: mole-fraction gradients of species 1, 2 per axis, except the x entry of an outlet node,
// which is replaced here by Eq. 37's -[B] J (J = imposed lattice flux).  Returns 1/tau per
// species; *hit is set when a clamp applied.
template <int DIMS>
__device__ inline void ms_relax(const StepArgs& a, double X0, double X1, double (&g0)[3],
                                double (&g1)[3], bool outlet, double& om0, double& om1, bool& hit)
{
    const double X2 = 1.0 - X0 - X1;
    // Eq. 32: B_ii = X_i / D_in + sum_{k != i} X_k / D_ik,  B_ij = -X_i (1/D_ij - 1/D_in)
    const double B00 = X0 * a.iD13 + X1 * a.iD12 + X2 * a.iD13;
    const double B01 = -X0 * (a.iD12 - a.iD13);
    const double B10 = -X1 * (a.iD12 - a.iD23);
    const double B11 = X1 * a.iD23 + X0 * a.iD12 + X2 * a.iD23;
    if (outlet) {
        g0[0] = -(B00 * a.Q0 + B01 * a.Q1);
        g1[0] = -(B10 * a.Q0 + B11 * a.Q1);
    }
    double n0 = 0.0, n1 = 0.0;
    if (a.ms_mode == 0) {
        // Eq. 34 with Gamma = I: J = -[B]^-1 grad X (Cramer's rule), then |J| per species
        const double det = B00 * B11 - B01 * B10;
        double q0 = 0.0, q1 = 0.0;
#pragma unroll
        for (int dd = 0; dd < DIMS; ++dd) {
            const double J0 = -(B11 * g0[dd] - B01 * g1[dd]) / det;
            const double J1 = -(B00 * g1[dd] - B10 * g0[dd]) / det;
            q0 += J0 * J0;
            q1 += J1 * J1;
        }
        n0 = sqrt(q0);
        n1 = sqrt(q1);
    }
    const double r21 = (a.ms_mode == 0) ? (n1 + a.eps1) / (n0 + a.eps0) : a.rst21;
    const double r12 = (a.ms_mode == 0) ? (n0 + a.eps0) / (n1 + a.eps1) : a.rst12;
    // Eq. 24 with N_i = sigma_i |N_i|; the inert species (sigma = 0) contributes X_3 / D_i3
    const double inv0 = (X1 - X0 * a.sgn12 * r21) * a.iD12 + X2 * a.iD13;
    const double inv1 = (X0 - X1 * a.sgn12 * r12) * a.iD12 + X2 * a.iD23;
    // Eq. 25 with c_s^2 = 1/3
    double t0 = 3.0 / inv0 + 0.5;
    double t1 = 3.0 / inv1 + 0.5;
    bool h = false;
    if (!(t0 >= a.tau_min)) { t0 = a.tau_min; h = true; }
    else if (t0 > a.tau_max) { t0 = a.tau_max; h = true; }
    if (!(t1 >= a.tau_min)) { t1 = a.tau_min; h = true; }
    else if (t1 > a.tau_max) { t1 = a.tau_max; h = true; }
    hit = h;
    om0 = 1.0 / t0;
    om1 = 1.0 / t1;
}

// central difference, one-sided next to a missing or solid neighbour, zero between two
__device__ inline double grad1(bool up, bool dn, double xu, double xc, double xd)
{
    if (up && dn) return 0.5 * (xu - xd);
    if (up) return xu - xc;
    if (dn) return xc - xd;
    return 0.0;
}

// BGK collision toward w_a X_s (Eq. 28-29) and store of the post-collision populations.
template <class L, int P, bool NS>
__device__ inline void collide_store(const StepArgs& a, long long n,
                                     typename Codec<P>::CT (&f)[2][L::Q], double X0, double X1,
                                     double om0, double om1)
{
    using C = Codec<P>;
    using CT = typename C::CT;
    using raw = typename C::raw;
    raw* __restrict__ fout = static_cast<raw*>(a.fout);
    const long long N = a.N;
    const CT o0 = (CT)om0, o1 = (CT)om1;
    const CT x0 = (CT)X0, x1 = (CT)X1;
    float c0 = (float)a.c0, c1 = (float)a.c1;
    if constexpr (NS) {
        c0 = (float)X0;
        c1 = (float)X1;
        a.xout[n] = c0;
        a.xout[N + n] = c1;
    }
#pragma unroll
    for (int k = 0; k < L::Q; ++k) {
        const CT wk = (CT)L::w[k];
        const CT v0 = f[0][k] + o0 * (wk * x0 - f[0][k]);
        const CT v1 = f[1][k] + o1 * (wk * x1 - f[1][k]);
        if constexpr (C::shifted) {
            const float wf = (float)L::w[k];
            fout[(long long)k * N + n] = C::enc(v0, wf * c0);
            fout[(long long)(L::Q + k) * N + n] = C::enc(v1, wf * c1);
        } else {
            fout[(long long)k * N + n] = C::enc(v0, CT(0));
            fout[(long long)(L::Q + k) * N + n] = C::enc(v1, CT(0));
        }
    }
}

}  // namespace lbmms
