// devmath.hpp -- device helpers of the relaxation step: constitutive laws in the H = F - I form,
// block reductions and the wavefront-wide affine scans of the damping pass.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

namespace tlsph {

template <typename R> __device__ __forceinline__ R rlog1p(R x);
template <> __device__ __forceinline__ float rlog1p<float>(float x) { return log1pf(x); }
template <> __device__ __forceinline__ double rlog1p<double>(double x) { return log1p(x); }
template <typename R> __device__ __forceinline__ R rsqrt_(R x);
template <> __device__ __forceinline__ float rsqrt_<float>(float x) { return sqrtf(x); }
template <> __device__ __forceinline__ double rsqrt_<double>(double x) { return sqrt(x); }

// det(I + H) - 1 without cancellation: tr H + (sum of principal 2x2 minors) + det H.
template <typename R, int D>
__device__ __forceinline__ R det_I_plus_H_minus_1(const R *H)
{
    if constexpr (D == 2) {
        return (H[0] + H[3]) + (H[0] * H[3] - H[1] * H[2]);
    } else {
        R tr = H[0] + H[4] + H[8];
        R m2 = (H[0] * H[4] - H[1] * H[3]) + (H[0] * H[8] - H[2] * H[6]) + (H[4] * H[8] - H[5] * H[7]);
        R d3 = H[0] * (H[4] * H[8] - H[5] * H[7]) - H[1] * (H[3] * H[8] - H[5] * H[6]) +
               H[2] * (H[3] * H[7] - H[4] * H[6]);
        return tr + m2 + d3;
    }
}

// Second Piola-Kirchhoff stress S of F = I + H from St Venant-Kirchhoff (Eq. 4) or neo-Hookean
// (Eqs. 7-8), written in H so that small strains keep their relative precision:
//   2E = H + H^T + H^T H,   C = I + 2E,
//   SVK: S = lambda tr(E) I + 2 mu E
//   NH:  S = mu (I - C^-1) + lambda ln J C^-1 = C^-1 (mu 2E + lambda ln J I),  ln J = log1p(J - 1)
// Also returns J - 1 and tr E.  Returns false when J <= 0 (neo-Hookean).
template <typename R, int D>
__device__ __forceinline__ bool stress_S(const R *H, int model, R lam, R mu, R *S, R &jm1, R &trE)
{
    R E2[D * D];
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
        for (int b = 0; b < D; ++b) {
            R s = H[a * D + b] + H[b * D + a];
#pragma unroll
            for (int k = 0; k < D; ++k) s += H[k * D + a] * H[k * D + b];
            E2[a * D + b] = s;
        }
    R tr = 0;
#pragma unroll
    for (int k = 0; k < D; ++k) tr += E2[k * D + k];
    trE = tr * R(0.5);
    jm1 = det_I_plus_H_minus_1<R, D>(H);
    bool ok = true;
    if (model == 0) {
#pragma unroll
        for (int a = 0; a < D; ++a)
#pragma unroll
            for (int b = 0; b < D; ++b) S[a * D + b] = mu * E2[a * D + b] + (a == b ? lam * trE : R(0));
    } else {
        ok = jm1 > R(-1);
        R lnJ = rlog1p<R>(ok ? jm1 : R(0));
        R J = R(1) + jm1;
        R detC = J * J;
        R C[D * D];
#pragma unroll
        for (int k = 0; k < D * D; ++k) C[k] = E2[k];
#pragma unroll
        for (int k = 0; k < D; ++k) C[k * D + k] += R(1);
        R Ci[D * D];
        if constexpr (D == 2) {
            Ci[0] = C[3] / detC; Ci[1] = -C[1] / detC; Ci[2] = -C[2] / detC; Ci[3] = C[0] / detC;
        } else {
            R inv = R(1) / detC;
            Ci[0] = (C[4] * C[8] - C[5] * C[7]) * inv;
            Ci[1] = (C[2] * C[7] - C[1] * C[8]) * inv;
            Ci[2] = (C[1] * C[5] - C[2] * C[4]) * inv;
            Ci[3] = (C[5] * C[6] - C[3] * C[8]) * inv;
            Ci[4] = (C[0] * C[8] - C[2] * C[6]) * inv;
            Ci[5] = (C[2] * C[3] - C[0] * C[5]) * inv;
            Ci[6] = (C[3] * C[7] - C[4] * C[6]) * inv;
            Ci[7] = (C[1] * C[6] - C[0] * C[7]) * inv;
            Ci[8] = (C[0] * C[4] - C[1] * C[3]) * inv;
        }
        R M[D * D];
#pragma unroll
        for (int k = 0; k < D * D; ++k) M[k] = mu * E2[k];
#pragma unroll
        for (int k = 0; k < D; ++k) M[k * D + k] += lam * lnJ;
#pragma unroll
        for (int a = 0; a < D; ++a)
#pragma unroll
            for (int b = 0; b < D; ++b) {
                R s = 0;
#pragma unroll
                for (int k = 0; k < D; ++k) s += Ci[a * D + k] * M[k * D + b];
                S[a * D + b] = s;
            }
    }
    return ok;
}

// P = F S = S + H S (Eq. 3).
template <typename R, int D>
__device__ __forceinline__ void piola(const R *H, const R *S, R *P)
{
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
        for (int b = 0; b < D; ++b) {
            R s = S[a * D + b];
#pragma unroll
            for (int k = 0; k < D; ++k) s += H[a * D + k] * S[k * D + b];
            P[a * D + b] = s;
        }
}

// T = P B0 with P = F S (Eq. 3), F = I + H.  Returns false when J <= 0 (neo-Hookean) or the
// result is not finite.
template <typename R, int D>
__device__ __forceinline__ bool stress_T(const R *H, const R *B0, int model, R lam, R mu, R *T)
{
    R S[D * D], P[D * D], jm1, trE;
    bool ok = stress_S<R, D>(H, model, lam, mu, S, jm1, trE);
    piola<R, D>(H, S, P);
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
        for (int b = 0; b < D; ++b) {
            R s = 0;
#pragma unroll
            for (int k = 0; k < D; ++k) s += P[a * D + k] * B0[k * D + b];
            T[a * D + b] = s;
            ok = ok && isfinite((double)s);
        }
    return ok;
}

// Von Mises stress of the Cauchy stress sigma = J^-1 P F^T (P = F S), sqrt(3/2 s:s) with s the
// deviator of the 3x3 sigma.  2D is plane strain (F33 = 1, E33 = 0): sigma33 = S33 / J with
// S33 = lambda tr E (SVK) or lambda ln J (neo-Hookean, C33 = 1).  NaN when J <= 0.
template <typename R, int D>
__device__ __forceinline__ R von_mises(const R *H, int model, R lam, R mu)
{
    R S[D * D], P[D * D], jm1, trE;
    const bool ok = stress_S<R, D>(H, model, lam, mu, S, jm1, trE);
    piola<R, D>(H, S, P);
    const R J = R(1) + jm1;
    const R rJ = R(1) / J;
    R sg[3][3];
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
        for (int b = 0; b < D; ++b) {
            // (P F^T)_ab = P_ab + sum_k P_ak H_bk
            R s = P[a * D + b];
#pragma unroll
            for (int k = 0; k < D; ++k) s += P[a * D + k] * H[b * D + k];
            sg[a][b] = s * rJ;
        }
    if constexpr (D == 2) {
        const R S33 = model == 0 ? lam * trE : lam * rlog1p<R>(jm1 > R(-1) ? jm1 : R(0));
        sg[0][2] = sg[1][2] = sg[2][0] = sg[2][1] = R(0);
        sg[2][2] = S33 * rJ;
    }
    const R d01 = sg[0][0] - sg[1][1], d12 = sg[1][1] - sg[2][2], d20 = sg[2][2] - sg[0][0];
    const R q = R(0.5) * (d01 * d01 + d12 * d12 + d20 * d20) +
                R(3) * (sg[0][1] * sg[0][1] + sg[1][2] * sg[1][2] + sg[0][2] * sg[0][2]);
    return (ok && J > R(0)) ? rsqrt_<R>(q) : R(NAN);
}

// Neumaier compensated addition in FP64.
__device__ __forceinline__ void neumaier(double &sum, double &comp, double x)
{
    double t = sum + x;
    if (fabs(sum) >= fabs(x))
        comp += (sum - t) + x;
    else
        comp += (x - t) + sum;
    sum = t;
}

}  // namespace tlsph
