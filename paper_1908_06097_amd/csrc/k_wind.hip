// Wind images from vorticity and divergence: the spectral step.
//
// On the unit sphere, with streamfunction psi and velocity potential chi
// (psi_n^m = -zeta_n^m / (n (n+1)), chi_n^m = -D_n^m / (n (n+1)), n >= 1), the
// wind images U = u cos(phi) = d chi/d lambda - (1 - mu^2) d psi/d mu and
// V = v cos(phi) = d psi/d lambda + (1 - mu^2) d chi/d mu are band-limited
// fields of truncation N + 1: d/d lambda multiplies a coefficient by i m, and
// with H_n^m = (1 - mu^2) dP̄_n^m/dmu = (n+1) eps_n^m P̄_{n-1}^m - n eps_{n+1}^m
// P̄_{n+1}^m, eps_n^m = sqrt((n^2 - m^2) / (4 n^2 - 1)), a sum over n of c_n H_n
// is the sum over k = m .. N+1 of P̄_k (k+2) eps_{k+1} c_{k+1} - (k-1) eps_k c_{k-1}.
// So
//   U_k^m = i m chi_k^m - [(k+2) eps_{k+1}^m psi_{k+1}^m - (k-1) eps_k^m psi_{k-1}^m]
//   V_k^m = i m psi_k^m + [(k+2) eps_{k+1}^m chi_{k+1}^m - (k-1) eps_k^m chi_{k-1}^m]
// and the grids follow from the ordinary inverse transform of truncation N + 1
// (the plan's own: its truncation is N + 1 and its fields are U then V).
#include "shtx_internal.h"

namespace shtx {

namespace {

template <typename T>
struct __attribute__((aligned(2 * sizeof(T)))) Cx {
    T x, y;
};

// One block per (m, field); threads over k = m .. N + 1.  vor, dvg are
// [F][nspec(N)], out [2F][nspec(N + 1)] (U of field f in row f, V in row F + f).
template <typename T>
__global__ void k_uv_spec(const Cx<T> *vor, const Cx<T> *dvg, Cx<T> *out, int N, int F)
{
    const int m = blockIdx.x, f = blockIdx.y;
    const int Tr = N + 1;
    const int64_t ns_in = (int64_t)(N + 1) * (N + 2) / 2, ns_out = (int64_t)(Tr + 1) * (Tr + 2) / 2;
    const int64_t in0 = (int64_t)f * ns_in + (int64_t)m * (2 * N + 3 - m) / 2;  // (m, n = m); m <= N only
    const int64_t out0 = (int64_t)m * (2 * Tr + 3 - m) / 2;
    Cx<T> *U = out + (int64_t)f * ns_out + out0;
    Cx<T> *V = out + (int64_t)(F + f) * ns_out + out0;
    // psi or chi of degree k (zero outside 1 <= k <= N and for m > N; Im of
    // the m = 0 coefficients ignored)
    auto pot = [&](const Cx<T> *a, int k) {
        Cx<T> r = {T(0), T(0)};
        if (m <= N && k >= m && k >= 1 && k <= N) {
            const Cx<T> z = a[in0 + (k - m)];
            const T sc = T(-1.0 / ((double)k * (k + 1)));
            r = Cx<T>{sc * z.x, m == 0 ? T(0) : sc * z.y};
        }
        return r;
    };
    auto eps = [&](int k) {
        return k <= m ? T(0) : T(sqrt(((double)k * k - (double)m * m) / (4.0 * k * k - 1.0)));
    };
    for (int k = m + (int)threadIdx.x; k <= Tr; k += blockDim.x) {
        const T ep = T(k + 2) * eps(k + 1), em = T(k - 1) * eps(k);
        const Cx<T> ps = pot(vor, k), ch = pot(dvg, k);
        const Cx<T> pu = pot(vor, k + 1), pd = pot(vor, k - 1);
        const Cx<T> cu = pot(dvg, k + 1), cd = pot(dvg, k - 1);
        const Cx<T> dps = {ep * pu.x - em * pd.x, ep * pu.y - em * pd.y};
        const Cx<T> dch = {ep * cu.x - em * cd.x, ep * cu.y - em * cd.y};
        const T mm = T(m);
        U[k - m] = Cx<T>{-mm * ch.y - dps.x, mm * ch.x - dps.y};
        V[k - m] = Cx<T>{-mm * ps.y + dch.x, mm * ps.x + dch.y};
    }
}

}  // namespace

hipError_t launch_uv_spec(const Plan &p, const void *vor, const void *dvg, void *out, hipStream_t s)
{
    // the plan's truncation is the winds' N + 1 and its fields are U then V
    if (p.trunc < 1 || p.nfld % 2 || !p.d_uvspec) return hipErrorInvalidValue;
    const int N = p.trunc - 1, F = p.nfld / 2;
    dim3 grid(p.trunc + 1, F);
    if (p.prec == SHTX_FP64)
        k_uv_spec<double><<<grid, 256, 0, s>>>((const Cx<double> *)vor, (const Cx<double> *)dvg, (Cx<double> *)out,
                                               N, F);
    else
        k_uv_spec<float><<<grid, 256, 0, s>>>((const Cx<float> *)vor, (const Cx<float> *)dvg, (Cx<float> *)out, N,
                                              F);
    return hipGetLastError();
}

}  // namespace shtx
