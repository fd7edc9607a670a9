// kuramoto_adjoint.hip - pathwise gradients of Kuramoto ensembles with
// respect to their parameters, for the parameter fitting that motivates the
// paper (Sec. 1.2).
//
// Objective of orbit o: R_o = (1/W) sum_{k = lo..hi} r(X^k), the order
// parameter of Eq. (7) averaged over a window of Euler-Maruyama iterates.
// With the noise path fixed (it is regenerated from the Philox counter, so
// forward and reverse passes see the same normals), the exact derivative of
// the discrete map follows from the adjoint recursion
//     lambda^N = w_N grad r(X^N);  for k = N-1 .. 0:
//         g        += (d Phi_k/d p)^T lambda^{k+1}
//         lambda^k  = (d Phi_k/d X)^T lambda^{k+1} + w_k grad r(X^k).
// For the Kuramoto map every product is O(N) through the phase sums
// C = sum cos X, S = sum sin X, A = sum lambda cos X, B = sum lambda sin X:
//     ((dPhi/dX)^T lambda)_j = lambda_j + kc (cos X_j A + sin X_j B
//                                            - lambda_j (cos X_j C + sin X_j S))
//     lambda^T dPhi/dK       = dt/N sum_i lambda_i (cos X_i S - sin X_i C)
//     lambda^T dPhi/domega_i = dt lambda_i,  lambda^T dPhi/dp_i = sqrt(dt) N_i lambda_i
//     d r/d X_j              = (S cos X_j - C sin X_j) / (N |Z|),  |Z| = sqrt(C^2 + S^2)
// (kc = K dt / N), which are the pairwise sums sum_i lambda_i cos(X_j - X_i)
// and sum_j sin(X_j - X_i) rewritten with the angle-difference identities.
//
// Memory: the forward pass stores every `every`-th state (checkpoints); the
// reverse pass walks the segments last to first, recomputes a segment's
// states from its checkpoint with the same em_step() as the forward pass,
// parks them with the normals of each step in a per-lane scratch area in
// HBM, and sweeps them backwards.
// The recomputed states are bitwise those of the forward pass: with
// compensation the forward pass carries each phase as hi + lo between
// checkpoints and restarts lo at 0 after writing one, exactly as a segment
// of the reverse pass starts from the stored hi.
// Parameter gradients are accumulated per lane in binary64; per-orbit rows
// are summed over orbits in binary64 in a fixed order, so the result does
// not depend on scheduling.
#include "kuramoto_lanes.hpp"
#include "launch.hpp"

namespace sode {
namespace {

using namespace kuramoto;

struct CkptArgs {
    const float* __restrict__ X0;
    const float* __restrict__ p;
    float* __restrict__ ckpt;
    double* __restrict__ R;
    int p_per_orbit;
    int compensated;
    int64_t orbits, every, nckpt, win_lo, win_hi;
    float dt, sqdt, dt_over_n;
    double inv_window;
    uint64_t seed, orbit_offset, step_offset;
};

struct AdjointArgs {
    const float* __restrict__ p;
    const float* __restrict__ ckpt;
    const double* __restrict__ dL_dR;
    float* __restrict__ seg;
    double* __restrict__ grad_rows;
    int p_per_orbit;
    int64_t orbits, every, nckpt, win_lo, win_hi;
    float dt, sqdt, dt_over_n, inv_window;
    double dt_d, sqdt_d;
    uint64_t seed, orbit_offset, step_offset;
};

__device__ __forceinline__ bool in_window(int64_t k, int64_t lo, int64_t hi) { return k >= lo && k <= hi; }

template <int N, bool COMP, bool MF>
__global__ __launch_bounds__(256) void forward_ckpt_kernel(const CkptArgs a)
{
    constexpr int P = N / 16;
    const int l = threadIdx.x & 15;
    const int64_t o = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 4;
    if (o >= a.orbits)
        return;
    const float* __restrict__ p = a.p + (a.p_per_orbit ? o * (int64_t)(2 * N + 1) : 0);
    const LaneCoefficients<P> c = lane_coefficients<P>(p, l, a.dt, a.sqdt, a.dt_over_n);
    const Stream st = orbit_stream(o, a.seed, a.orbit_offset, nullptr, nullptr);
    float* __restrict__ ck = a.ckpt + o * a.nckpt * N + P * l;

    float th[P], tl[P];
#pragma unroll
    for (int i = 0; i < P; ++i) {
        th[i] = load_phase(a.X0[o * N + P * l + i]);
        tl[i] = 0.0f;
        ck[i] = th[i];
    }
    // Statistic accumulated in binary64 (every lane holds the row's value).
    double racc = in_window(0, a.win_lo, a.win_hi) ? (double)order_parameter<P>(th) : 0.0;
    if constexpr (P <= 2) {
        // Normals of B = 4/P steps at a time, one Philox block per quad or
        // pair of lanes and step (lane_normals_steps).
        constexpr int B = 4 / P;
        const int64_t nsteps = (a.nckpt - 1) * a.every;
        int64_t cidx = 1, to_ckpt = a.every;
        for (int64_t j = 0; j < nsteps; j += B) {
            float xb[B][P];
            lane_normals_steps<P>(st, (uint32_t)(a.step_offset + (uint64_t)j), l, xb);
#pragma unroll
            for (int t = 0; t < B; ++t) {
                const int64_t k = j + t;
                if (t == 0 || k < nsteps) {
                    em_step<P, COMP, MF>(th, tl, c, st, (uint32_t)(a.step_offset + (uint64_t)k), l, nullptr, xb[t]);
                    if (in_window(k + 1, a.win_lo, a.win_hi))
                        racc += (double)order_parameter<P>(th);
                    if (--to_ckpt == 0) {
#pragma unroll
                        for (int i = 0; i < P; ++i) {
                            ck[cidx * N + i] = th[i];
                            tl[i] = 0.0f;  // a checkpoint is an exact restart point
                        }
                        ++cidx;
                        to_ckpt = a.every;
                    }
                }
            }
        }
    } else {
        int64_t k = 0;
        for (int64_t cidx = 1; cidx < a.nckpt; ++cidx) {
            for (int64_t kk = 0; kk < a.every; ++kk, ++k) {
                em_step<P, COMP, MF>(th, tl, c, st, (uint32_t)(a.step_offset + (uint64_t)k), l);
                if (in_window(k + 1, a.win_lo, a.win_hi))
                    racc += (double)order_parameter<P>(th);
            }
#pragma unroll
            for (int i = 0; i < P; ++i) {
                ck[cidx * N + i] = th[i];
                tl[i] = 0.0f;  // a checkpoint is an exact restart point
            }
        }
    }
    if (l == 0)
        a.R[o] = racc * a.inv_window;
}

// lambda += w grad r(X), from the row sums C, S and the lane's cos/sin.
template <int P>
__device__ __forceinline__ void add_window_seed(float (&lam)[P], const float (&cs)[P], const float (&sn)[P],
                                                float C, float S, float w)
{
    constexpr float kInvN = 1.0f / (float)(16 * P);
    const float z = __builtin_sqrtf(C * C + S * S);
    if (z >= 1e-30f) {
        const float scale = w * kInvN / z;
#pragma unroll
        for (int i = 0; i < P; ++i)
            lam[i] += scale * (S * cs[i] - C * sn[i]);
    }
}

// Sum of a binary64 value over the 16 lanes of a row.
__device__ __forceinline__ double row_sum_f64(double v)
{
#pragma unroll
    for (int m = 8; m >= 1; m >>= 1)
        v += __shfl_xor(v, m, 16);
    return v;
}

template <int N, bool COMP, bool MF>
__global__ __launch_bounds__(256) void adjoint_kernel(const AdjointArgs a)
{
    constexpr int P = N / 16;
    const int l = threadIdx.x & 15;
    const int64_t o = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 4;
    if (o >= a.orbits)
        return;
    const float* __restrict__ p = a.p + (a.p_per_orbit ? o * (int64_t)(2 * N + 1) : 0);
    const LaneCoefficients<P> c = lane_coefficients<P>(p, l, a.dt, a.sqdt, a.dt_over_n);
    const Stream st = orbit_stream(o, a.seed, a.orbit_offset, nullptr, nullptr);
    const float* __restrict__ ck = a.ckpt + o * a.nckpt * N + P * l;
    // Scratch layout [orbit][step in segment][lane][2P]: a lane's P phases
    // X^k followed by the P normals of step k, so the reverse sweep does not
    // draw the normals again; a row's 16 lanes write and read 32 P
    // consecutive floats per step.
    float* __restrict__ seg = a.seg + (o * a.every * 16 + l) * (2 * P);
    const int64_t nsteps = (a.nckpt - 1) * a.every;

    float lam[P];
    double gK = 0.0, gW[P], gS[P];
#pragma unroll
    for (int i = 0; i < P; ++i) {
        lam[i] = 0.0f;
        gW[i] = 0.0;
        gS[i] = 0.0;
    }
    if (in_window(nsteps, a.win_lo, a.win_hi)) {
        float th[P], cs[P], sn[P], C, S;
#pragma unroll
        for (int i = 0; i < P; ++i)
            th[i] = ck[(a.nckpt - 1) * N + i];
        phase_sums<P>(th, cs, sn, C, S);
        add_window_seed<P>(lam, cs, sn, C, S, a.inv_window);
    }

    for (int64_t cidx = a.nckpt - 2; cidx >= 0; --cidx) {
        const int64_t kbase = cidx * a.every;
        // Recompute the segment's states X^{kbase} .. X^{kbase+every-1}.
        float th[P], tl[P];
#pragma unroll
        for (int i = 0; i < P; ++i) {
            th[i] = ck[cidx * N + i];
            tl[i] = 0.0f;
        }
        if constexpr (P <= 2) {
            constexpr int B = 4 / P;
            for (int64_t j0 = 0; j0 < a.every; j0 += B) {
                float xb[B][P];
                lane_normals_steps<P>(st, (uint32_t)(a.step_offset + (uint64_t)(kbase + j0)), l, xb);
#pragma unroll
                for (int t = 0; t < B; ++t) {
                    const int64_t j = j0 + t;
                    if (t == 0 || j < a.every) {
                        float* __restrict__ rec = seg + j * 16 * (2 * P);
#pragma unroll
                        for (int i = 0; i < P; ++i)
                            rec[i] = th[i];
                        if (j + 1 < a.every)
                            em_step<P, COMP, MF>(th, tl, c, st, (uint32_t)(a.step_offset + (uint64_t)(kbase + j)), l,
                                                 rec + P, xb[t]);
                    }
                }
            }
        } else {
            for (int64_t j = 0; j < a.every; ++j) {
                float* __restrict__ rec = seg + j * 16 * (2 * P);
#pragma unroll
                for (int i = 0; i < P; ++i)
                    rec[i] = th[i];
                if (j + 1 < a.every)
                    em_step<P, COMP, MF>(th, tl, c, st, (uint32_t)(a.step_offset + (uint64_t)(kbase + j)), l,
                                         rec + P);
            }
        }
        // Reverse sweep over the segment.  The record of step j - 1 is
        // loaded while step j is processed, off the dependency chain.
        float nX[P], nxi[P];
        {
            const float* __restrict__ rec = seg + (a.every - 1) * 16 * (2 * P);
#pragma unroll
            for (int i = 0; i < P; ++i)
                nX[i] = rec[i];
            // The segment's last step was not taken by the recompute.
            lane_normals<P>(st, (uint32_t)(a.step_offset + (uint64_t)(kbase + a.every - 1)), l, nxi);
        }
        for (int64_t j = a.every - 1; j >= 0; --j) {
            const int64_t k = kbase + j;
            float X[P], xi[P], cs[P], sn[P], C, S;
#pragma unroll
            for (int i = 0; i < P; ++i) {
                X[i] = nX[i];
                xi[i] = nxi[i];
            }
            if (j > 0) {
                const float* __restrict__ rec = seg + (j - 1) * 16 * (2 * P);
#pragma unroll
                for (int i = 0; i < P; ++i) {
                    nX[i] = rec[i];
                    nxi[i] = rec[P + i];
                }
            }
            phase_sums<P>(X, cs, sn, C, S);
            float la = 0.0f, lb = 0.0f, kpart = 0.0f;
#pragma unroll
            for (int i = 0; i < P; ++i) {
                la += lam[i] * cs[i];
                lb += lam[i] * sn[i];
                kpart += lam[i] * (cs[i] * S - sn[i] * C);
                gW[i] += (double)lam[i];
                gS[i] += (double)(xi[i] * lam[i]);
            }
            gK += (double)kpart;
            const float A = row_sum(la), B = row_sum(lb);
#pragma unroll
            for (int i = 0; i < P; ++i)
                lam[i] += c.kc[0] * (cs[i] * A + sn[i] * B - lam[i] * (cs[i] * C + sn[i] * S));
            if (in_window(k, a.win_lo, a.win_hi))
                add_window_seed<P>(lam, cs, sn, C, S, a.inv_window);
        }
    }

    gK = row_sum_f64(gK);
    const double wgt = a.dL_dR ? a.dL_dR[o] : 1.0;
    double* __restrict__ row = a.grad_rows + o * (int64_t)(2 * N + 1);
    if (l == 0)
        row[0] = wgt * gK * (a.dt_d / (double)N);
#pragma unroll
    for (int i = 0; i < P; ++i) {
        row[1 + P * l + i] = wgt * gW[i] * a.dt_d;
        row[1 + N + P * l + i] = wgt * gS[i] * a.sqdt_d;
    }
}

// grad[q] = sum_o rows[o][q] in binary64: a strided per-thread sum in orbit
// order followed by a fixed LDS tree, one block per parameter.
__global__ __launch_bounds__(256) void sum_rows_kernel(const double* __restrict__ rows, int64_t orbits,
                                                       int d, double* __restrict__ grad)
{
    __shared__ double part[256];
    const int q = blockIdx.x;
    double acc = 0.0;
    for (int64_t o = threadIdx.x; o < orbits; o += 256)
        acc += rows[o * d + q];
    part[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            part[threadIdx.x] += part[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        grad[q] = part[0];
}

template <int N>
hipError_t launch_ckpt_n(const AdjointRequest& r)
{
    CkptArgs a;
    a.X0 = static_cast<const float*>(r.X0);
    a.p = static_cast<const float*>(r.p);
    a.ckpt = static_cast<float*>(r.ckpt);
    a.R = r.R;
    a.p_per_orbit = r.p_per_orbit;
    a.compensated = r.compensated;
    a.orbits = r.orbits;
    a.every = r.every;
    a.nckpt = r.nsteps / r.every + 1;
    a.win_lo = r.win_lo;
    a.win_hi = r.win_hi;
    a.dt = (float)r.dt;
    a.sqdt = (float)sqrt(r.dt);
    a.dt_over_n = (float)(r.dt / (double)N);
    a.inv_window = 1.0 / (double)(r.win_hi - r.win_lo + 1);
    a.seed = r.seed;
    a.orbit_offset = r.orbit_offset;
    a.step_offset = r.step_offset;
    const dim3 grid((unsigned)((r.orbits * 16 + 255) / 256));
    const bool mf = r.drift == 1;
    if (r.compensated && mf)
        hipLaunchKernelGGL((forward_ckpt_kernel<N, true, true>), grid, dim3(256), 0, r.stream, a);
    else if (r.compensated)
        hipLaunchKernelGGL((forward_ckpt_kernel<N, true, false>), grid, dim3(256), 0, r.stream, a);
    else if (mf)
        hipLaunchKernelGGL((forward_ckpt_kernel<N, false, true>), grid, dim3(256), 0, r.stream, a);
    else
        hipLaunchKernelGGL((forward_ckpt_kernel<N, false, false>), grid, dim3(256), 0, r.stream, a);
    return hipGetLastError();
}

template <int N>
hipError_t launch_adjoint_n(const AdjointRequest& r)
{
    AdjointArgs a;
    a.p = static_cast<const float*>(r.p);
    a.ckpt = static_cast<const float*>(r.ckpt);
    a.dL_dR = r.dL_dR;
    a.seg = r.seg_scratch;
    a.grad_rows = r.grad_rows;
    a.p_per_orbit = r.p_per_orbit;
    a.orbits = r.orbits;
    a.every = r.every;
    a.nckpt = r.nsteps / r.every + 1;
    a.win_lo = r.win_lo;
    a.win_hi = r.win_hi;
    a.dt = (float)r.dt;
    a.sqdt = (float)sqrt(r.dt);
    a.dt_over_n = (float)(r.dt / (double)N);
    a.inv_window = (float)(1.0 / (double)(r.win_hi - r.win_lo + 1));
    a.dt_d = r.dt;
    a.sqdt_d = sqrt(r.dt);
    a.seed = r.seed;
    a.orbit_offset = r.orbit_offset;
    a.step_offset = r.step_offset;
    if (r.orbits > 0) {
        const dim3 grid((unsigned)((r.orbits * 16 + 255) / 256));
        const bool mf = r.drift == 1;
        if (r.compensated && mf)
            hipLaunchKernelGGL((adjoint_kernel<N, true, true>), grid, dim3(256), 0, r.stream, a);
        else if (r.compensated)
            hipLaunchKernelGGL((adjoint_kernel<N, true, false>), grid, dim3(256), 0, r.stream, a);
        else if (mf)
            hipLaunchKernelGGL((adjoint_kernel<N, false, true>), grid, dim3(256), 0, r.stream, a);
        else
            hipLaunchKernelGGL((adjoint_kernel<N, false, false>), grid, dim3(256), 0, r.stream, a);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return e;
    }
    if (r.grad) {
        hipLaunchKernelGGL(sum_rows_kernel, dim3(2 * N + 1), dim3(256), 0, r.stream, r.grad_rows, r.orbits,
                           2 * N + 1, r.grad);
        return hipGetLastError();
    }
    return hipSuccess;
}

}  // namespace

hipError_t launch_kuramoto_forward_ckpt_f32(const AdjointRequest& r)
{
    switch (r.n) {
    case 16: return launch_ckpt_n<16>(r);
    case 32: return launch_ckpt_n<32>(r);
    case 64: return launch_ckpt_n<64>(r);
    case 128: return launch_ckpt_n<128>(r);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_kuramoto_adjoint_f32(const AdjointRequest& r)
{
    switch (r.n) {
    case 16: return launch_adjoint_n<16>(r);
    case 32: return launch_adjoint_n<32>(r);
    case 64: return launch_adjoint_n<64>(r);
    case 128: return launch_adjoint_n<128>(r);
    default: return hipErrorInvalidValue;
    }
}

bool adjoint_supports(int n) { return n == 16 || n == 32 || n == 64 || n == 128; }

}  // namespace sode
