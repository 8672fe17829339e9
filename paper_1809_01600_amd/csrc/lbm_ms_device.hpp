// Device-side building blocks of one time step of the LBM / Maxwell-Stefan method
// (arXiv 1809.01600): velocity sets, population storage codecs, the pull with its boundary
// rules, and the FP64 Maxwell-Stefan relaxation-time solve.
#pragma once

#include <hip/hip_runtime.h>
#include <type_traits>
#include <stdint.h>

namespace lbmms {

// ---------------------------------------------------------------------------------------------
// neighbour bits returned by the pull (which axis neighbours exist and are fluid)
// ---------------------------------------------------------------------------------------------
constexpr uint32_t NB_XM = 1u << 0;  // x - 1
constexpr uint32_t NB_XP = 1u << 1;  // x + 1
constexpr uint32_t NB_YM = 1u << 2;  // y - 1 (periodic)
constexpr uint32_t NB_YP = 1u << 3;
constexpr uint32_t NB_ZM = 1u << 4;  // z - 1 (periodic)
constexpr uint32_t NB_ZP = 1u << 5;

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
    // FP32 weights whose exact sum is one (the nearest floats to 4/9, 1/9, 1/36 sum to 1 + 7.5e-9,
    // and a collision toward w_a X in float would then create that fraction of X at every node off
    // equilibrium, a bias in the steady state): 1/9 and 1/36 in units of 2^-27, the rest weight
    // the remainder in units of 2^-25, each within 6e-8 of its weight
    static constexpr long long M1 = ((1LL << 27) + 4) / 9, M2 = ((1LL << 27) + 18) / 36;
    static constexpr float W0F = (float)((double)((1LL << 25) - M1 - M2) / (double)(1LL << 25));
    static constexpr float W1F = (float)((double)M1 / (double)(1LL << 27));
    static constexpr float W2F = (float)((double)M2 / (double)(1LL << 27));
    static constexpr float wf[9] = {W0F, W1F, W1F, W1F, W1F, W2F, W2F, W2F, W2F};
};

// D2Q5, named beside D2Q9 in Sec. 2.3: rest and the four axis links in Eq. 2's order, weights
// 1/3 and 1/6, the same second moment c_s^2 = 1/3 with five populations instead of nine.
struct D2Q5 {
    static constexpr int Q = 5;
    static constexpr int DIMS = 2;
    static constexpr int ex[5] = {0, 1, 0, -1, 0};
    static constexpr int ey[5] = {0, 0, 1, 0, -1};
    static constexpr int ez[5] = {0, 0, 0, 0, 0};
    static constexpr int opp[5] = {0, 3, 4, 1, 2};
    static constexpr double w[5] = {1.0 / 3, 1.0 / 6, 1.0 / 6, 1.0 / 6, 1.0 / 6};
    // FP32 weights with an exact unit sum: 1/6 rounded to float, the rest weight 1 - 4 w1 (a
    // multiple of 2^-24 in [1/4, 1/2), so itself a float)
    static constexpr float W1F = (float)(1.0 / 6);
    static constexpr float W0F = (float)(1.0 - 4.0 * (double)W1F);
    static constexpr float wf[5] = {W0F, W1F, W1F, W1F, W1F};
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
    // FP32 weights whose exact sum is one (the nearest floats sum to 1 + 1.5e-8): 1/18 in units of
    // 2^-28, 1/36 in units of 2^-29 taken at the next value below it with M1 + M2 divisible by 4,
    // so that the remainder 1 - 6 w1 - 12 w2, the rest weight, is a float; each within 1.3e-7 of
    // its weight
    static constexpr long long M1 = ((1LL << 28) + 9) / 18, R2 = ((1LL << 29) + 18) / 36;
    static constexpr long long M2 = R2 - (M1 + R2) % 4;
    static constexpr float W0F = (float)((double)((1LL << 28) - 6 * M1 - 6 * M2) / (double)(1LL << 28));
    static constexpr float W1F = (float)((double)M1 / (double)(1LL << 28));
    static constexpr float W2F = (float)((double)M2 / (double)(1LL << 29));
    static constexpr float wf[19] = {W0F, W1F, W1F, W1F, W1F, W1F, W1F, W2F, W2F, W2F,
                                     W2F, W2F, W2F, W2F, W2F, W2F, W2F, W2F, W2F};
};

// D3Q7: rest and the six axis links.  c_s^2 = 1/3 (Sec. 3.1) makes the axis weight 1/6 and the
// rest weight 0.
struct D3Q7 {
    static constexpr int Q = 7;
    static constexpr int DIMS = 3;
    static constexpr int ex[7] = {0, 1, -1, 0, 0, 0, 0};
    static constexpr int ey[7] = {0, 0, 0, 1, -1, 0, 0};
    static constexpr int ez[7] = {0, 0, 0, 0, 0, 1, -1};
    static constexpr int opp[7] = {0, 2, 1, 4, 3, 6, 5};
    static constexpr double w[7] = {0.0, 1.0 / 6, 1.0 / 6, 1.0 / 6, 1.0 / 6, 1.0 / 6, 1.0 / 6};
    // FP32 weights with an exact unit sum and all six axis weights equal: 1/6 rounded down to a
    // multiple of 2^-25, and the remainder 1 - 6 w1 = 2^-24 on the rest link
    static constexpr long long M1 = (1LL << 25) / 6;
    static constexpr float W1F = (float)((double)M1 / (double)(1LL << 25));
    static constexpr float W0F = (float)((double)((1LL << 25) - 6 * M1) / (double)(1LL << 25));
    static constexpr float wf[7] = {W0F, W1F, W1F, W1F, W1F, W1F, W1F};
};

// sum of the weights of the links with e_x = +1 (1/6 for every set)
constexpr double W_OUT = 1.0 / 6.0;

// Sum of a float weight table in FP64 (exact: every entry is a multiple of 2^-29 below one) and
// the check that the rest weight survived its cast to float.
template <class L>
constexpr double wf_sum()
{
    double t = 0.0;
    for (int k = 0; k < L::Q; ++k) t += (double)L::wf[k];
    return t;
}
static_assert(wf_sum<D2Q9>() == 1.0 && wf_sum<D3Q19>() == 1.0 && wf_sum<D2Q5>() == 1.0 &&
                  wf_sum<D3Q7>() == 1.0,
              "float weights must sum to one");
static_assert((double)D3Q7::W1F * (1LL << 25) == (double)D3Q7::M1 &&
                  (double)D3Q7::W0F * (1LL << 25) == (double)((1LL << 25) - 6 * D3Q7::M1),
              "D3Q7 weights are not floats");
static_assert((double)D2Q5::W0F == 1.0 - 4.0 * (double)D2Q5::W1F, "D2Q5 rest weight is not a float");
static_assert((double)D2Q9::W0F * (1LL << 25) == (double)((1LL << 25) - D2Q9::M1 - D2Q9::M2),
              "D2Q9 rest weight is not a float");
static_assert((double)D3Q19::W0F * (1LL << 28) == (double)((1LL << 28) - 6 * D3Q19::M1 - 6 * D3Q19::M2),
              "D3Q19 rest weight is not a float");

// Weight of link k in the arithmetic type CT: the FP64 weights, or the float table above.
template <class L, class CT>
__host__ __device__ constexpr CT wgt(int k)
{
    if constexpr (sizeof(CT) == sizeof(double)) return (CT)L::w[k];
    else return L::wf[k];
}

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
// 16-bit storage of the shifted population h = f - s (s = w_a c).  FP16 stores h * 2^12: the
// power of two is exact, so normal values round exactly as unscaled ones would, while the small
// deviations of the NODE shift (1e-8 to 1e-4 on long, weakly graded domains) stay clear of FP16's
// subnormal range (below 6.1e-5), where they would lose most of their bits.  |h| <= 1 for mole
// fractions, so h * 2^12 <= 4096 stays far inside FP16's range.
template <> struct Codec<P_F16> {
    using raw = _Float16;
    using CT = float;
    static constexpr bool shifted = true;
    static constexpr float SCALE = 4096.f, INV = 1.f / 4096.f;
    __device__ static inline CT dec(raw r, CT s) { return (float)r * INV + s; }
    __device__ static inline raw enc(CT v, CT s) { return (_Float16)((v - s) * SCALE); }
};
template <> struct Codec<P_BF16> {
    using raw = __bf16;
    using CT = float;
    static constexpr bool shifted = true;
    __device__ static inline CT dec(raw r, CT s) { return (float)r + s; }
    __device__ static inline raw enc(CT v, CT s) { return (__bf16)(v - s); }
};

// ---------------------------------------------------------------------------------------------
// global-memory accessors: uniform base pointer + 32-bit byte offset (global_load/store with an
// SGPR base and a VGPR offset; the pointers come from an in-memory table, so without the explicit
// address space the compiler would fall back to flat accesses)
// ---------------------------------------------------------------------------------------------
#define LBMMS_GLOBAL __attribute__((address_space(1)))
template <class T>
__device__ inline T gload(const void* base, unsigned byte_off)
{
    return *(const LBMMS_GLOBAL T*)((const LBMMS_GLOBAL char*)base + byte_off);
}
template <class T>
__device__ inline void gstore(void* base, unsigned byte_off, T v)
{
    *(LBMMS_GLOBAL T*)((LBMMS_GLOBAL char*)base + byte_off) = v;
}
// a store marked non-temporal: the line is not kept in the L2 for reuse
template <class T>
__device__ inline void gstore_nt(void* base, unsigned byte_off, T v)
{
    __builtin_nontemporal_store(v, (LBMMS_GLOBAL T*)((LBMMS_GLOBAL char*)base + byte_off));
}

// ---------------------------------------------------------------------------------------------
// per-launch arguments
// ---------------------------------------------------------------------------------------------
struct StepArgs {
    const void* fin;          // post-collision populations of step t   [Q][P][2] (fluid nodes)
    void* fout;               // post-collision populations of step t+1 [Q][P][2]
    const double* xin;        // node reference c of step t   [2][NF] (NODE shift only)
    double* xout;             // node reference c of step t+1 [2][NF]
    const int* idx;           // dense [N]: compact fluid index of the node, -1 for solid
    unsigned* flags;          // [0]: relaxation time clamped
    long long N;              // nodes of the box
    long long NF;             // fluid nodes
    long long P;              // elements between consecutive (species, link) planes (>= NF)
    int nx, ny, nz;
    int tiles_x, tiles_y, chunks_z;
    double iD12, iD13, iD23;  // 1 / D*_ij (lattice units)
    double Xin0, Xin1;        // inlet mole fractions (Dirichlet rule, Eq. 36)
    double Q0, Q1;            // lattice outflow per open outlet node (Eq. 39 scaled)
    double eps0, eps1;        // eps * |nu_1|, eps * |nu_2| (flux-norm regularizer)
    double sgn12;             // sigma_1 * sigma_2, sigma_i = -sgn(nu_i) (Eq. 24 sign rule)
    double rst21, rst12;      // stoichiometric ratios |nu_2|/|nu_1|, |nu_1|/|nu_2|
    double c0, c1;            // global shift composition (16-bit GLOBAL storage)
    double om_lo, om_hi;      // 1 / tau_max, 1 / tau_min (relaxation-time clamp)
    int ms_mode;              // 0 local flux norms, 1 stoichiometric ratio
    int inlet_wall;           // 1: x = 0 face is a bounce-back wall
    double S0, S1;            // volumetric source per fluid node and step (Eq. 27) ...
    int src_x0;               // ... on the columns x >= src_x0 (nx: none)
    int trt;                  // 1: two-relaxation-time collision
    double trt_lambda;        // (tau_even - 1/2)(tau - 1/2)
};

// Population layout: the two evolved species of one (link, node) pair side by side,
// [link][node][species] (P nodes per link), so that one 2-element load or store moves both: a
// pull issues Q memory instructions per node instead of 2Q.  pop_node: byte offset of node m in
// link 0; pop_link: bytes between links; pop_spec: bytes between the two species of a pair.
// With LBMMS_SOA the plain layout [species][link][P] is used instead.
#ifdef LBMMS_SOA
template <unsigned ES>
__device__ inline unsigned pop_node(unsigned m) { return m * ES; }
template <unsigned ES>
__device__ inline unsigned pop_link(const StepArgs& a) { return (unsigned)a.P * ES; }
template <class L, unsigned ES>
__device__ inline unsigned pop_spec(const StepArgs& a) { return (unsigned)L::Q * (unsigned)a.P * ES; }
template <class L>
__device__ inline long long pop_elem(const StepArgs& a, int j, long long i) { return (long long)j * a.P + i; }
#else
template <unsigned ES>
__device__ inline unsigned pop_node(unsigned m) { return m * (2u * ES); }
template <unsigned ES>
__device__ inline unsigned pop_link(const StepArgs& a) { return (unsigned)a.P * (2u * ES); }
template <class L, unsigned ES>
__device__ inline unsigned pop_spec(const StepArgs& a) { (void)a; return ES; }
// element index of population j = s Q + k (species s, link k) of node i
template <class L>
__device__ inline long long pop_elem(const StepArgs& a, int j, long long i)
{
    const int s = j >= L::Q ? 1 : 0;
    return ((long long)(j - s * L::Q) * a.P + i) * 2 + s;
}
#endif

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
// Source of link a is r - e_a (periodic in y and z).  Links whose source is solid bounce back
// (f_a(r) = f*_abar(r)); at the outlet column the links from x = nx take the exact-flux rule
// f_a = f*_abar - (w_abar / W_out) Q_s; at the inlet column the links from x = -1 take
// f_a = (w_a + w_abar) X_in - f_abar (Eq. 36) with f_abar the value just pulled, or bounce back
// when the inlet is a wall.
//
// Source slots: si[a] = compact index of the source node, -1 if it is solid, BOUNDARY for the
// links that cross the inlet or outlet face.
constexpr int BOUNDARY = -3;

// neighbour bit of an axis link whose source is fluid
template <class L>
__device__ inline uint32_t axis_bit(int k, int s)
{
    const int ex = L::ex[k], ey = L::ey[k], ez = L::ez[k];
    if (s < 0) return 0u;
    if (ey == 0 && ez == 0 && ex != 0) return ex == 1 ? NB_XM : NB_XP;
    if (ex == 0 && ez == 0 && ey != 0) return ey == 1 ? NB_YM : NB_YP;
    if (ex == 0 && ey == 0 && ez != 0) return ez == 1 ? NB_ZM : NB_ZP;
    return 0u;
}

// Source slots from the dense index map in global memory.
template <class L>
__device__ inline uint32_t global_sources(const StepArgs& a, int x, int y, int z, long long n, int i,
                                          int (&si)[L::Q])
{
    const long long nx = a.nx;
    const long long plane = nx * a.ny;
    const long long oym = (y > 0) ? -nx : (long long)(a.ny - 1) * nx;
    const long long oyp = (y < a.ny - 1) ? nx : -(long long)(a.ny - 1) * nx;
    const long long ozm = (z > 0) ? -plane : (long long)(a.nz - 1) * plane;
    const long long ozp = (z < a.nz - 1) ? plane : -(long long)(a.nz - 1) * plane;
    uint32_t nb = 0;
#pragma unroll
    for (int k = 0; k < L::Q; ++k) {
        const int ex = L::ex[k], ey = L::ey[k], ez = L::ez[k];
        if (k == 0) { si[k] = i; continue; }
        if ((ex == -1 && x == a.nx - 1) || (ex == 1 && x == 0)) { si[k] = BOUNDARY; continue; }
        long long src = n - ex;
        if (ey == 1) src += oym;
        if (ey == -1) src += oyp;
        if (ez == 1) src += ozm;
        if (ez == -1) src += ozp;
        si[k] = gload<int>(a.idx, (unsigned)src * 4u);
        nb |= axis_bit<L>(k, si[k]);
    }
    return nb;
}

// Branch-free gather of the post-stream populations of compact node i from its source slots,
// then the inlet rule and the moments.  A lane with nothing to do passes i = 0 and zero slots.
//
// NODE shift: a stored post-collision population is f*_a = w_a c + h_a, with c an FP64 reference
// per node and species and h_a in the storage precision.  The slowest mode of a steady solve
// lives in the moment X, so X is carried in FP64 and only the small deviations h_a are rounded:
// for the links of node i, dc_a = c(source) - c(i) and h_a are small, X = c(i) + sum_a (w_a dc_a
// + h_a), and the output is g_a = f_a - w_a X = w_a (dc_a - S) + h_a with S = X - c(i).
// Where the references c come from: global memory by compact index, or an LDS-staged copy of the
// region around the node (position pos, row pitch RX).
struct RefGlobal {
    const double* xin;
    unsigned xsp;  // bytes per species
    __device__ inline double own(int s, int i) const { return gload<double>(xin, (unsigned)i * 8u + s * xsp); }
    template <class L>
    __device__ inline double src(int s, int k, unsigned m) const { return gload<double>(xin, m * 8u + s * xsp); }
};
template <int RX, int RY>
struct RefLds {
    const double* sc;  // [2][RY * RX]
    int pos;
    __device__ inline double own(int s, int) const { return sc[s * RY * RX + pos]; }
    template <class L>
    __device__ inline double src(int s, int k, unsigned) const
    {
        return sc[s * RY * RX + pos - L::ey[k] * RX - L::ex[k]];
    }
};

// LDS-staged references of a ring of NPL planes ([plane slot][species][RY * RX]); the node sits
// at column cx, row cy of relative plane zr (slot (zr + 2) % NPL).
template <int RX, int RY, int NPL>
struct RefLds3 {
    const double* sc;
    int zr, pos;
    __device__ inline double own(int s, int) const
    {
        return sc[((((zr + 2) % NPL + NPL) % NPL) * 2 + s) * RY * RX + pos];
    }
    template <class L>
    __device__ inline double src(int s, int k, unsigned) const
    {
        const int slot = ((zr - L::ez[k] + 2) % NPL + NPL) % NPL;
        return sc[(slot * 2 + s) * RY * RX + pos - L::ey[k] * RX - L::ex[k]];
    }
};

template <class L, int P, class REF>
__device__ inline void gather_ns(const StepArgs& a, int i, const int (&si)[L::Q], bool inlet,
                                 bool outlet, float (&g)[2][L::Q], double& X0, double& X1,
                                 const REF& ref)
{
    using C = Codec<P>;
    using raw = typename C::raw;
    constexpr unsigned ES = sizeof(raw);
    const void* fin = a.fin;
    const unsigned plane = pop_link<ES>(a);
    const unsigned spec = pop_spec<L, ES>(a);
    const double co0 = ref.own(0, i);
    const double co1 = ref.own(1, i);
    const bool wall = a.inlet_wall != 0;
    float dc[2][L::Q];
#pragma unroll
    for (int k = 0; k < L::Q; ++k) {
        const int ex = L::ex[k];
        const bool from_out = (ex == -1) && outlet;
        const bool from_in = (ex == 1) && inlet;
        const int s = si[k];
        const bool local = (s < 0) || from_out || from_in;
        const bool reflect = (s == -1) || from_out || (from_in && wall);
        const unsigned m = (unsigned)(local ? i : s);
        const unsigned off = (reflect ? (unsigned)L::opp[k] : (unsigned)k) * plane + pop_node<ES>(m);
        g[0][k] = C::dec(gload<raw>(fin, off), 0.f);
        g[1][k] = C::dec(gload<raw>(fin, off + spec), 0.f);
        dc[0][k] = local ? 0.f : (float)(ref.template src<L>(0, k, m) - co0);
        dc[1][k] = local ? 0.f : (float)(ref.template src<L>(1, k, m) - co1);
        if (L::ex[k] == -1) {
            const float frac = (float)(L::w[L::opp[k]] / W_OUT);
            g[0][k] = from_out ? g[0][k] - frac * (float)a.Q0 : g[0][k];
            g[1][k] = from_out ? g[1][k] - frac * (float)a.Q1 : g[1][k];
        }
    }
    // Eq. 36: f_a = 2 w_a X_in - f_abar, i.e. reference 2 X_in - c_abar and deviation -h_abar
    const bool anti = inlet && !wall;
    const float di0 = (float)(2.0 * (a.Xin0 - co0)), di1 = (float)(2.0 * (a.Xin1 - co1));
#pragma unroll
    for (int k = 0; k < L::Q; ++k) {
        if (L::ex[k] == 1) {
            const int o = L::opp[k];
            dc[0][k] = anti ? di0 - dc[0][o] : dc[0][k];
            dc[1][k] = anti ? di1 - dc[1][o] : dc[1][k];
            g[0][k] = anti ? -g[0][o] : g[0][k];
            g[1][k] = anti ? -g[1][o] : g[1][k];
        }
    }
    // the sum of small terms: FP64 for FP32 deviations; FP32 for 16-bit ones, whose own rounding
    // (about 1e-3 of each term) dwarfs that of an FP32 sum.  The weights here are the nearest
    // floats, not the unit-sum table: they multiply reference differences and so shape the
    // diffusion operator, while the FP64 reference already makes the node update conservative.
    using AT = typename std::conditional<P == P_F32, double, float>::type;
    AT S0 = 0, S1 = 0;
#pragma unroll
    for (int k = 0; k < L::Q; ++k) {
        S0 += (AT)((float)L::w[k] * dc[0][k]) + (AT)g[0][k];
        S1 += (AT)((float)L::w[k] * dc[1][k]) + (AT)g[1][k];
    }
    X0 = co0 + (double)S0;
    X1 = co1 + (double)S1;
    const float s0 = (float)S0, s1 = (float)S1;
#pragma unroll
    for (int k = 0; k < L::Q; ++k) {
        g[0][k] += (float)L::w[k] * (dc[0][k] - s0);
        g[1][k] += (float)L::w[k] * (dc[1][k] - s1);
    }
}

// The plain gather in two halves, so that a caller can issue the loads of several nodes before
// it waits for any of them: gather_issue loads the raw stored values each link pulls (the source
// entry, or this node's own opposite entry where it reflects), gather_finish decodes them,
// applies the outlet flux share and the inlet rule (Eq. 36), and sums the moments.
template <class L, int P>
__device__ inline void gather_issue(const StepArgs& a, int i, const int (&si)[L::Q], bool inlet,
                                    bool outlet, typename Codec<P>::raw (&r)[2][L::Q])
{
    using raw = typename Codec<P>::raw;
    constexpr unsigned ES = sizeof(raw);
    const void* fin = a.fin;
    const unsigned plane = pop_link<ES>(a);             // bytes between links
    const unsigned spec = pop_spec<L, ES>(a);           // ... and between the two species
    const bool wall = a.inlet_wall != 0;
#pragma unroll
    for (int k = 0; k < L::Q; ++k) {
        const int ex = L::ex[k];
        const bool from_out = (ex == -1) && outlet;
        const bool from_in = (ex == 1) && inlet;
        const int s = si[k];
        const bool local = (s < 0) || from_out || from_in;  // read this node's own entry
        const bool reflect = (s == -1) || from_out || (from_in && wall);
        const unsigned m = (unsigned)(local ? i : s);
        const unsigned off = (reflect ? (unsigned)L::opp[k] : (unsigned)k) * plane + pop_node<ES>(m);
        r[0][k] = gload<raw>(fin, off);
        r[1][k] = gload<raw>(fin, off + spec);
    }
}

template <class L, int P>
__device__ inline void gather_finish(const StepArgs& a, const typename Codec<P>::raw (&r)[2][L::Q],
                                     bool inlet, bool outlet, typename Codec<P>::CT (&f)[2][L::Q],
                                     double& X0, double& X1)
{
    using C = Codec<P>;
    using CT = typename C::CT;
    const float cg0 = (float)a.c0, cg1 = (float)a.c1;
    const bool wall = a.inlet_wall != 0;
#pragma unroll
    for (int k = 0; k < L::Q; ++k) {
        const bool from_out = (L::ex[k] == -1) && outlet;
        if constexpr (C::shifted) {
            const float wk = L::wf[k];  // w of the opposite link is the same
            f[0][k] = C::dec(r[0][k], wk * cg0);
            f[1][k] = C::dec(r[1][k], wk * cg1);
        } else {
            f[0][k] = C::dec(r[0][k], CT(0));
            f[1][k] = C::dec(r[1][k], CT(0));
        }
        if (L::ex[k] == -1) {
            const CT frac = (CT)(L::w[L::opp[k]] / W_OUT);
            f[0][k] = from_out ? f[0][k] - frac * (CT)a.Q0 : f[0][k];
            f[1][k] = from_out ? f[1][k] - frac * (CT)a.Q1 : f[1][k];
        }
    }
    const bool anti = inlet && !wall;
#pragma unroll
    for (int k = 0; k < L::Q; ++k) {
        if (L::ex[k] == 1) {
            const CT ww = (CT)(L::w[k] + L::w[L::opp[k]]);
            f[0][k] = anti ? ww * (CT)a.Xin0 - f[0][L::opp[k]] : f[0][k];
            f[1][k] = anti ? ww * (CT)a.Xin1 - f[1][L::opp[k]] : f[1][k];
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

template <class L, int P, bool NS>
__device__ inline void gather(const StepArgs& a, int i, const int (&si)[L::Q], bool inlet,
                              bool outlet, typename Codec<P>::CT (&f)[2][L::Q], double& X0,
                              double& X1)
{
    if constexpr (NS) {
        gather_ns<L, P>(a, i, si, inlet, outlet, f, X0, X1, RefGlobal{a.xin, (unsigned)a.NF * 8u});
        return;
    } else {
        typename Codec<P>::raw r[2][L::Q];
        gather_issue<L, P>(a, i, si, inlet, outlet, r);
        gather_finish<L, P>(a, r, inlet, outlet, f, X0, X1);
    }
}

// Pull of node (x, y, z) (dense n, compact i) through the global index map; returns NB_* bits.
template <class L, int P, bool NS>
__device__ inline uint32_t pull_node(const StepArgs& a, int x, int y, int z, long long n, int i,
                                     typename Codec<P>::CT (&f)[2][L::Q], double& X0, double& X1)
{
    int si[L::Q];
    const uint32_t nb = global_sources<L>(a, x, y, z, n, i, si);
    gather<L, P, NS>(a, i, si, x == 0, x == a.nx - 1, f, X0, X1);
    return nb;
}

// 1/d in FP64 from the hardware reciprocal estimate and two Newton steps (each doubles the
// number of correct bits), without the scaling and fix-up of a correctly rounded division; the
// operands here are positive and far from the denormal and overflow ranges.
__device__ inline double rcp64(double d)
{
    double r = __builtin_amdgcn_rcp(d);
    r = r * (2.0 - d * r);
    r = r * (2.0 - d * r);
    return r;
}

// ---------------------------------------------------------------------------------------------
// Maxwell-Stefan flux solve and relaxation times (FP64)
// ---------------------------------------------------------------------------------------------
// g0/g1: mole-fraction gradients of species 1, 2 per axis, except the x entry of an outlet node,
// which is replaced here by Eq. 37's -[B] J (J = imposed lattice flux).  Returns 1/tau per
// species; *hit is set when a clamp applied.
// The node's Maxwell-Stefan matrix [B] (Eq. 32) and, with RDET and the local flux-norm ratio,
// the reciprocal of its determinant: everything of the solve that the gradients do not enter.
struct MsMat {
    double B00, B01, B10, B11, rdet;
};

// The clamp of tau to [tau_min, tau_max], applied to w = 1/tau: a tau below tau_min, a negative
// one included (1/D in (-6, 0) gives w < 0), becomes tau_min, and one above tau_max becomes
// tau_max; a non-finite w counts as below tau_min.  Sets h when it applies.
__device__ inline double clamp_omega(const StepArgs& a, double w, bool& h)
{
    if (!(w <= a.om_hi) || __builtin_signbit(w)) {
        h = true;
        return a.om_hi;
    }
    if (w < a.om_lo) {
        h = true;
        return a.om_lo;
    }
    return w;
}

template <bool RDET>
__device__ inline MsMat ms_matrix(const StepArgs& a, double X0, double X1)
{
    const double X2 = 1.0 - X0 - X1;
    MsMat m;
    // Eq. 32: B_ii = X_i / D_in + sum_{k != i} X_k / D_ik,  B_ij = -X_i (1/D_ij - 1/D_in)
    m.B00 = X0 * a.iD13 + X1 * a.iD12 + X2 * a.iD13;
    m.B01 = -X0 * (a.iD12 - a.iD13);
    m.B10 = -X1 * (a.iD12 - a.iD23);
    m.B11 = X1 * a.iD23 + X0 * a.iD12 + X2 * a.iD23;
    m.rdet = 0.0;
    if (RDET && a.ms_mode == 0) m.rdet = rcp64(m.B00 * m.B11 - m.B01 * m.B10);
    return m;
}

template <int DIMS, bool RDET>
__device__ inline void ms_relax(const StepArgs& a, double X0, double X1, const MsMat& m,
                                double (&g0)[3], double (&g1)[3], bool outlet, double& om0,
                                double& om1, bool& hit)
{
    const double X2 = 1.0 - X0 - X1;
    const double B00 = m.B00, B01 = m.B01, B10 = m.B10, B11 = m.B11;
    if (outlet) {
        g0[0] = -(B00 * a.Q0 + B01 * a.Q1);
        g1[0] = -(B10 * a.Q0 + B11 * a.Q1);
    }
    double n0 = 0.0, n1 = 0.0;
    if (a.ms_mode == 0) {
        // Eq. 34 with Gamma = I: J = -[B]^-1 grad X (Cramer's rule), then |J| per species
        const double rdet = RDET ? m.rdet : rcp64(B00 * B11 - B01 * B10);
        double q0 = 0.0, q1 = 0.0;
#pragma unroll
        for (int dd = 0; dd < DIMS; ++dd) {
            const double J0 = -(B11 * g0[dd] - B01 * g1[dd]) * rdet;
            const double J1 = -(B00 * g1[dd] - B10 * g0[dd]) * rdet;
            q0 += J0 * J0;
            q1 += J1 * J1;
        }
        n0 = sqrt(q0);
        n1 = sqrt(q1);
    }
    double r21 = a.rst21, r12 = a.rst12;
    if (a.ms_mode == 0) {
        // flux-norm ratios |N_2|/|N_1| and |N_1|/|N_2| through one reciprocal
        const double u = n1 + a.eps1, v = n0 + a.eps0;
        const double ruv = rcp64(u * v);
        r21 = u * u * ruv;
        r12 = v * v * ruv;
    }
    // Eq. 24 with N_i = sigma_i |N_i|; the inert species (sigma = 0) contributes X_3 / D_i3
    const double inv0 = (X1 - X0 * a.sgn12 * r21) * a.iD12 + X2 * a.iD13;
    const double inv1 = (X0 - X1 * a.sgn12 * r12) * a.iD12 + X2 * a.iD23;
    // Eq. 25 with c_s^2 = 1/3: tau = 3 D + 1/2, so 1/tau = (1/D) / (3 + (1/D) / 2), clamped
    bool h = false;
    om0 = clamp_omega(a, inv0 * rcp64(3.0 + 0.5 * inv0), h);
    om1 = clamp_omega(a, inv1 * rcp64(3.0 + 0.5 * inv1), h);
    hit = h;
}

template <int DIMS>
__device__ inline void ms_relax(const StepArgs& a, double X0, double X1, double (&g0)[3],
                                double (&g1)[3], bool outlet, double& om0, double& om1, bool& hit)
{
    ms_relax<DIMS, false>(a, X0, X1, ms_matrix<false>(a, X0, X1), g0, g1, outlet, om0, om1, hit);
}

// central difference, one-sided next to a missing or solid neighbour, zero between two
__device__ inline double grad1(bool up, bool dn, double xu, double xc, double xd)
{
    if (up && dn) return 0.5 * (xu - xd);
    if (up) return xu - xc;
    if (dn) return xc - xd;
    return 0.0;
}

// BGK collision toward w_a X_s (Eq. 28-29) plus the source term w_a S_s of Eq. 27 (s0, s1; zero
// off the reaction layer), and store of the post-collision populations.  The source enters as
// a shift of the equilibrium: f + omega (w X - f) + w S = f + omega (w (X + S / omega) - f).
// NODE shift: f holds g_a = f_a - w_a X, so f*_a = w_a (X + S) + (1 - omega) g_a; the deviations
// are rounded to the storage precision and the node reference c = X + S - sum_a h_a (FP64)
// keeps the stored moment equal to X + S whatever the rounding.  NT: global-shift stores marked
// non-temporal (the compacted 3D columns, whose next plane re-reads lines the L2 would otherwise
// give up to the stores).
template <class L, int P, bool NS, bool NT = false>
__device__ inline void collide_store(const StepArgs& a, int n,
                                     typename Codec<P>::CT (&f)[2][L::Q], double X0, double X1,
                                     double om0, double om1, double s0, double s1)
{
    using C = Codec<P>;
    using CT = typename C::CT;
    using raw = typename C::raw;
    constexpr unsigned ES = sizeof(raw);
    void* fout = a.fout;
    const unsigned plane = pop_link<ES>(a);
    const unsigned spec = pop_spec<L, ES>(a);
    const unsigned base = pop_node<ES>((unsigned)n);
    // TRT: the odd part of a link pair relaxes with omega (it carries the flux, so Eq. 25 still
    // sets D); the even part with omega_e = 1 / (1/2 + Lambda / (1/omega - 1/2))
    double oe0 = om0, oe1 = om1;
    if (a.trt) {
        const double h0 = 1.0 - 0.5 * om0, h1 = 1.0 - 0.5 * om1;
        oe0 = h0 * rcp64(0.5 * h0 + a.trt_lambda * om0);
        oe1 = h1 * rcp64(0.5 * h1 + a.trt_lambda * om1);
    }
    // a workgroup-uniform branch: the BGK loops carry no TRT terms
    auto store = [&](auto trt_tag) {
        constexpr bool TRT = decltype(trt_tag)::value;
        if constexpr (NS) {
            const float k0 = (float)(1.0 - om0), k1 = (float)(1.0 - om1);
            const float d0 = (float)(0.5 * (om0 - oe0)), d1 = (float)(0.5 * (om1 - oe1));
            using AT = typename std::conditional<P == P_F32, double, float>::type;
            AT sh0 = 0, sh1 = 0;
#pragma unroll
            for (int k = 0; k < L::Q; ++k) {
                // TRT: h = g - omega_e (g + g_bar) / 2 - omega (g - g_bar) / 2
                //        = (1 - omega) g + d (g + g_bar),  d = (omega - omega_e) / 2
                float h0 = k0 * f[0][k], h1 = k1 * f[1][k];
                if constexpr (TRT) {
                    const int o = L::opp[k];
                    h0 += d0 * (f[0][k] + f[0][o]);
                    h1 += d1 * (f[1][k] + f[1][o]);
                }
                const raw r0 = C::enc(h0, 0.f);
                const raw r1 = C::enc(h1, 0.f);
                sh0 += (AT)C::dec(r0, 0.f);
                sh1 += (AT)C::dec(r1, 0.f);
                const unsigned off = base + (unsigned)k * plane;
                gstore<raw>(fout, off, r0);
                gstore<raw>(fout, off + spec, r1);
            }
            gstore<double>(a.xout, (unsigned)n * 8u, X0 + s0 - (double)sh0);
            gstore<double>(a.xout, (unsigned)n * 8u + (unsigned)a.NF * 8u, X1 + s1 - (double)sh1);
        } else {
            double Y0 = X0, Y1 = X1;
            if (s0 != 0.0 || s1 != 0.0) {  // only on the reaction layer; the source is even
                Y0 += s0 * rcp64(oe0);
                Y1 += s1 * rcp64(oe1);
            }
            const CT o0 = (CT)om0, o1 = (CT)om1;
            const CT x0 = (CT)Y0, x1 = (CT)Y1;
            const CT d0 = (CT)(0.5 * (om0 - oe0)), d1 = (CT)(0.5 * (om1 - oe1));
            const float c0 = (float)a.c0, c1 = (float)a.c1;
#pragma unroll
            for (int k = 0; k < L::Q; ++k) {
                const CT wk = wgt<L, CT>(k);
                CT v0 = f[0][k] + o0 * (wk * x0 - f[0][k]);
                CT v1 = f[1][k] + o1 * (wk * x1 - f[1][k]);
                if constexpr (TRT) {
                    // f - omega_e (f_even - w x) - omega f_odd = BGK + d (f + f_bar - 2 w x)
                    const int o = L::opp[k];
                    v0 += d0 * (f[0][k] + f[0][o] - (CT)2 * wk * x0);
                    v1 += d1 * (f[1][k] + f[1][o] - (CT)2 * wk * x1);
                }
                const unsigned off = base + (unsigned)k * plane;
                if constexpr (C::shifted) {
                    const float wf = L::wf[k];
                    gstore<raw>(fout, off, C::enc(v0, wf * c0));
                    gstore<raw>(fout, off + spec, C::enc(v1, wf * c1));
                } else if constexpr (NT) {
                    gstore_nt<raw>(fout, off, C::enc(v0, CT(0)));
                    gstore_nt<raw>(fout, off + spec, C::enc(v1, CT(0)));
                } else {
                    gstore<raw>(fout, off, C::enc(v0, CT(0)));
                    gstore<raw>(fout, off + spec, C::enc(v1, CT(0)));
                }
            }
        }
    };
    if (a.trt)
        store(std::true_type{});
    else
        store(std::false_type{});
}

}  // namespace lbmms
