// Advective coupling (Sec. 3.1: Eq. 20-21, the Eq. 26 equilibrium with the molar-averaged
// velocity u_M, and a second lattice Boltzmann model for u_M).  When the electrode reaction changes
// the number of moles (nu_1 + nu_2 != 0) the total flux N_t = C_t u_M no longer vanishes, and the
// species relax toward w_a X_s (1 + e_a . u_M / c_s^2).  u_M comes from a velocity model whose
// density is the total concentration (normalized to one), taken in its Stokes limit: equilibrium
// w_a (rho + 3 e_a . u), u = sum_a e_a g_a, BGK with 1 / tau_flow; no-slip half-way bounce-back on
// solid, the inlet at rho = 1 (anti-bounce-back) and each open outlet node carrying the
// electrode's total molar flux Q_t = Q_1 + Q_2 (the exact-flux rule of the species).  The species
// see the mean node velocity of this step and the last, which removes the velocity model's
// undamped period-2 mode (populations at equilibrium, so untouched by any collision, whose node
// velocity alternates in space and time while every link flux stays uniform).
//
// Eq. 24 with advection takes the diffusive fluxes of Eq. 20, J_s = N_s - X_s N_t (the populations
// carry the advective part through Eq. 26), so the inert species has J_3 = -J_1 - J_2.  The ratio
// J_j / J_i of two flux vectors is their projection (J_j . J_i) / |J_i|^2, pulled toward the
// one-dimensional steady ratio (Nh_j - X_j Nh_t) / (Nh_i - X_i Nh_t) with Nh_s = -nu_s by the
// regularizer eps; the stoichiometric variant uses that ratio alone.  Eq. 37's outlet-column
// gradient takes the diffusive boundary flux J_s = Q_s - X_s Q_t.
//
// Two passes per step over the fluid nodes of the box (one thread per voxel, grid-stride): the
// first pulls the species and writes X (FP64) per compact node; the second pulls both models
// again, reads the neighbours' X for the gradients and does the rest.  FP64 and FP32 storage,
// global (unshifted) storage; every lattice.
#include <hip/hip_runtime.h>

#include "lbm_ms_kernels.hpp"

namespace lbmms {

namespace {

inline int adv_grid(long long n)
{
    long long g = (n + 255) / 256;
    return (int)(g < 1 ? 1 : (g > 65535 ? 65535 : g));
}

__device__ inline void voxel_xyz(const StepArgs& a, long long n, int& x, int& y, int& z)
{
    x = (int)(n % a.nx);
    y = (int)((n / a.nx) % a.ny);
    z = (int)(n / ((long long)a.nx * a.ny));
}

// Pull of the velocity model's populations of node i from its source slots (the species' slots):
// stream, half-way bounce-back on solid, the inlet at rho = 1 and the outlet flux Q_t.
template <class L, int P>
__device__ inline void flow_gather(const StepArgs& a, const AdvArgs& v, int i, const int (&si)[L::Q],
                                   bool inlet, bool outlet, typename Codec<P>::CT (&g)[L::Q])
{
    using C = Codec<P>;
    using CT = typename C::CT;
    using raw = typename C::raw;
    constexpr unsigned ES = sizeof(raw);
    const unsigned plane = (unsigned)a.P * ES;
#pragma unroll
    for (int k = 0; k < L::Q; ++k) {
        const int ex = L::ex[k];
        const bool from_out = (ex == -1) && outlet;
        const bool from_in = (ex == 1) && inlet;
        const int s = si[k];
        const bool local = (s < 0) || from_out || from_in;
        const bool reflect = (s == -1) || from_out;
        const unsigned m = (unsigned)(local ? i : s);
        const unsigned off = (reflect ? (unsigned)L::opp[k] : (unsigned)k) * plane + m * ES;
        g[k] = C::dec(gload<raw>(v.gin, off), CT(0));
        if (from_out) g[k] -= (CT)(L::w[L::opp[k]] / W_OUT) * (CT)v.Qt;
    }
#pragma unroll
    for (int k = 0; k < L::Q; ++k)
        if (L::ex[k] == 1 && inlet) g[k] = (CT)(L::w[k] + L::w[L::opp[k]]) - g[L::opp[k]];
}

// Eq. 24-25 with the diffusive fluxes; g0/g1 are the gradients (the x entry of an outlet node is
// replaced by Eq. 37's -[B] J with J_s = Q_s - X_s Q_t).  Returns 1 / tau per species.
template <int DIMS>
__device__ inline void ms_relax_adv(const StepArgs& a, const AdvArgs& v, double X0, double X1,
                                    double (&g0)[3], double (&g1)[3], bool outlet, double& om0,
                                    double& om1, bool& hit)
{
    const double X[3] = {X0, X1, 1.0 - X0 - X1};
    const MsMat m = ms_matrix<false>(a, X0, X1);
    if (outlet) {
        const double J0 = a.Q0 - X0 * v.Qt, J1 = a.Q1 - X1 * v.Qt;
        g0[0] = -(m.B00 * J0 + m.B01 * J1);
        g1[0] = -(m.B10 * J0 + m.B11 * J1);
    }
    const double det = m.B00 * m.B11 - m.B01 * m.B10;
    double J[3][3];
#pragma unroll
    for (int d = 0; d < DIMS; ++d) {
        J[0][d] = -(m.B11 * g0[d] - m.B01 * g1[d]) / det;
        J[1][d] = -(m.B00 * g1[d] - m.B10 * g0[d]) / det;
        J[2][d] = -J[0][d] - J[1][d];
    }
    const double nh[3] = {v.nh0, v.nh1, v.nh2};
    // 1 / D*_ij for the pairs (0,1), (0,2), (1,2)
    const double iD[3][3] = {{0.0, a.iD12, a.iD13}, {a.iD12, 0.0, a.iD23}, {a.iD13, a.iD23, 0.0}};
    double w[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        double inv = 0.0;
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            if (j == i) continue;
            double r = (nh[j] - X[j] * v.nht) / (nh[i] - X[i] * v.nht);
            if (a.ms_mode == 0) {
                double dot = 0.0, nn = 0.0;
#pragma unroll
                for (int d = 0; d < DIMS; ++d) {
                    dot += J[j][d] * J[i][d];
                    nn += J[i][d] * J[i][d];
                }
                r = (dot + v.eps2 * r) / (nn + v.eps2);
            }
            inv += (X[j] - X[i] * r) * iD[i][j];
        }
        // Eq. 25: tau = 3 D + 1/2, i.e. 1 / tau = (1/D) / (3 + (1/D) / 2)
        w[i] = inv / (3.0 + 0.5 * inv);
    }
    bool h = false;
    om0 = clamp_omega(a, w[0], h);
    om1 = clamp_omega(a, w[1], h);
    hit = h;
}

}  // namespace

// pass 1: X of every fluid node (species pull with its boundary rules).  Both passes run one
// thread per fluid node (vox gives its voxel), so no lane idles on a solid voxel.
template <class L, int P>
__global__ __launch_bounds__(256) void k_adv_moments(StepArgs a, const int* __restrict__ vox, double* xw)
{
    using CT = typename Codec<P>::CT;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < a.NF;
         i += (long long)gridDim.x * blockDim.x) {
        const long long n = vox[i];
        int x, y, z;
        voxel_xyz(a, n, x, y, z);
        CT f[2][L::Q];
        double X0, X1;
        pull_node<L, P, false>(a, x, y, z, n, i, f, X0, X1);
        xw[i] = X0;
        xw[a.NF + i] = X1;
    }
}

// pass 2: the coupled step of every fluid node
template <class L, int P>
__global__ __launch_bounds__(256) void k_adv_step(StepArgs a, AdvArgs v)
{
    using C = Codec<P>;
    using CT = typename C::CT;
    using raw = typename C::raw;
    constexpr unsigned ES = sizeof(raw);
    const unsigned plane = (unsigned)a.P * ES;             // velocity model: [Q][P]
    const unsigned link = pop_link<ES>(a);                   // species: the population layout
    const unsigned spec = pop_spec<L, ES>(a);
    for (long long ii = blockIdx.x * (long long)blockDim.x + threadIdx.x; ii < a.NF;
         ii += (long long)gridDim.x * blockDim.x) {
        const int i = (int)ii;
        const long long n = v.vox[i];
        int x, y, z;
        voxel_xyz(a, n, x, y, z);
        int si[L::Q];
        global_sources<L>(a, x, y, z, n, i, si);
        const bool inlet = x == 0, outlet = x == a.nx - 1;
        CT f[2][L::Q];
        double X0, X1;
        gather<L, P, false>(a, i, si, inlet, outlet, f, X0, X1);
        CT g[L::Q];
        flow_gather<L, P>(a, v, i, si, inlet, outlet, g);
        double rho = 0.0, u[3] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int k = 0; k < L::Q; ++k) {
            const double gk = (double)g[k];
            rho += gk;
            u[0] += L::ex[k] * gk;
            u[1] += L::ey[k] * gk;
            u[2] += L::ez[k] * gk;
        }
        // gradients from the neighbours' X: the source of the axis link +e_d is r - e_d, of -e_d
        // r + e_d (solid and beyond-face sources are not fluid: one-sided, Eq. 35 at the inlet)
        double g0[3] = {0.0, 0.0, 0.0}, g1[3] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int kp = 1; kp < L::Q; ++kp) {
            const int d = L::ex[kp] == 1 ? 0 : (L::ey[kp] == 1 ? 1 : (L::ez[kp] == 1 ? 2 : -1));
            if (d < 0 || L::ex[kp] + L::ey[kp] + L::ez[kp] != 1 ||
                L::ex[kp] * L::ex[kp] + L::ey[kp] * L::ey[kp] + L::ez[kp] * L::ez[kp] != 1)
                continue;
            const int sd = si[kp], su = si[L::opp[kp]];
            const bool fd = sd >= 0, fu = su >= 0;
            const double xd0 = fd ? v.xc[sd] : 0.0, xd1 = fd ? v.xc[a.NF + sd] : 0.0;
            const double xu0 = fu ? v.xc[su] : 0.0, xu1 = fu ? v.xc[a.NF + su] : 0.0;
            g0[d] = grad1(fu, fd, xu0, X0, xd0);
            g1[d] = grad1(fu, fd, xu1, X1, xd1);
        }
        double om0, om1;
        bool hit;
        ms_relax_adv<L::DIMS>(a, v, X0, X1, g0, g1, outlet, om0, om1, hit);
        if (hit) gstore<unsigned>(a.flags, 0u, 1u);
        // the species see the two-step mean velocity
        double um[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const long long ui = (long long)d * a.NF + i;
            um[d] = 0.5 * (u[d] + v.uin[ui]);
            v.uout[ui] = u[d];
        }
        const CT o0 = (CT)om0, o1 = (CT)om1, of = (CT)v.om_flow;
        const CT x0 = (CT)X0, x1 = (CT)X1, r = (CT)rho;
        const unsigned base = (unsigned)i * ES;
        const unsigned sbase = pop_node<ES>((unsigned)i);
#pragma unroll
        for (int k = 0; k < L::Q; ++k) {
            const CT wk = wgt<L, CT>(k);
            const CT em = (CT)(3.0 * (L::ex[k] * um[0] + L::ey[k] * um[1] + L::ez[k] * um[2]));
            const CT eu = (CT)(3.0 * (L::ex[k] * u[0] + L::ey[k] * u[1] + L::ez[k] * u[2]));
            const CT s0 = f[0][k] + o0 * (wk * x0 * ((CT)1 + em) - f[0][k]);
            const CT s1 = f[1][k] + o1 * (wk * x1 * ((CT)1 + em) - f[1][k]);
            const CT gg = g[k] + of * (wk * (r + eu) - g[k]);
            const unsigned off = sbase + (unsigned)k * link;
            gstore<raw>(a.fout, off, C::enc(s0, CT(0)));
            gstore<raw>(a.fout, off + spec, C::enc(s1, CT(0)));
            gstore<raw>(v.gout, base + (unsigned)k * plane, C::enc(gg, CT(0)));
        }
    }
}

// velocity model at rest (rho = 1, u = 0) and zero node velocities of both parities
template <class L, int P>
__global__ __launch_bounds__(256) void k_adv_rest(StepArgs a, AdvArgs v, double* u_other)
{
    using C = Codec<P>;
    using CT = typename C::CT;
    using raw = typename C::raw;
    raw* gout = static_cast<raw*>(v.gout);
    for (long long n = blockIdx.x * (long long)blockDim.x + threadIdx.x; n < a.N;
         n += (long long)gridDim.x * blockDim.x) {
        const int i = a.idx[n];
        if (i < 0) continue;
#pragma unroll
        for (int k = 0; k < L::Q; ++k) gout[(long long)k * a.P + i] = C::enc(wgt<L, CT>(k), CT(0));
        for (int d = 0; d < 3; ++d) {
            v.uout[(long long)d * a.NF + i] = 0.0;
            u_other[(long long)d * a.NF + i] = 0.0;
        }
    }
}

// u_M the species see, [3][N] (solid 0), times `scale` (lattice to physical units)
template <class L, int P>
__global__ __launch_bounds__(256) void k_adv_velocity(StepArgs a, const double* ucur,
                                                      const double* uprev, double scale,
                                                      double* out)
{
    for (long long n = blockIdx.x * (long long)blockDim.x + threadIdx.x; n < a.N;
         n += (long long)gridDim.x * blockDim.x) {
        const int i = a.idx[n];
        for (int d = 0; d < 3; ++d) {
            const long long ui = (long long)d * a.NF + i;
            out[(long long)d * a.N + n] = i < 0 ? 0.0 : 0.5 * (ucur[ui] + uprev[ui]) * scale;
        }
    }
}

template <class L, int P>
static hipError_t adv_step_l(hipStream_t st, const StepArgs& a, const AdvArgs& v, double* xw)
{
    hipLaunchKernelGGL((k_adv_moments<L, P>), dim3(adv_grid(a.NF)), dim3(256), 0, st, a, v.vox, xw);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_adv_step<L, P>), dim3(adv_grid(a.NF)), dim3(256), 0, st, a, v);
    return hipGetLastError();
}

template <class L, int P>
static hipError_t adv_rest_l(hipStream_t st, const StepArgs& a, const AdvArgs& v, double* u_other)
{
    hipLaunchKernelGGL((k_adv_rest<L, P>), dim3(adv_grid(a.N)), dim3(256), 0, st, a, v, u_other);
    return hipGetLastError();
}

template <class L, int P>
static hipError_t adv_velocity_l(hipStream_t st, const StepArgs& a, const double* ucur,
                                 const double* uprev, double scale, double* out)
{
    hipLaunchKernelGGL((k_adv_velocity<L, P>), dim3(adv_grid(a.N)), dim3(256), 0, st, a, ucur,
                       uprev, scale, out);
    return hipGetLastError();
}

#define LBMMS_ADV_DISPATCH(FN, ...)                                                               \
    do {                                                                                         \
        if (prec != P_F64 && prec != P_F32) return hipErrorInvalidValue;                         \
        const bool f64 = prec == P_F64;                                                          \
        switch (lattice) {                                                                       \
        case 0: return f64 ? FN<D2Q9, P_F64>(__VA_ARGS__) : FN<D2Q9, P_F32>(__VA_ARGS__);         \
        case 1: return f64 ? FN<D3Q19, P_F64>(__VA_ARGS__) : FN<D3Q19, P_F32>(__VA_ARGS__);       \
        case 2: return f64 ? FN<D2Q5, P_F64>(__VA_ARGS__) : FN<D2Q5, P_F32>(__VA_ARGS__);         \
        case 3: return f64 ? FN<D3Q7, P_F64>(__VA_ARGS__) : FN<D3Q7, P_F32>(__VA_ARGS__);         \
        }                                                                                        \
        return hipErrorInvalidValue;                                                             \
    } while (0)

hipError_t launch_adv_step(hipStream_t st, const StepArgs& a, const AdvArgs& v, double* xw,
                           int lattice, int prec)
{
    LBMMS_ADV_DISPATCH(adv_step_l, st, a, v, xw);
}

hipError_t launch_adv_rest(hipStream_t st, const StepArgs& a, const AdvArgs& v, double* u_other,
                           int lattice, int prec)
{
    LBMMS_ADV_DISPATCH(adv_rest_l, st, a, v, u_other);
}

hipError_t launch_adv_velocity(hipStream_t st, const StepArgs& a, const double* ucur,
                               const double* uprev, double scale, double* out, int lattice,
                               int prec)
{
    LBMMS_ADV_DISPATCH(adv_velocity_l, st, a, ucur, uprev, scale, out);
}

#undef LBMMS_ADV_DISPATCH

}  // namespace lbmms
