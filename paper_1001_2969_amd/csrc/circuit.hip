// External circuit of the powered electrode (Sec. 2.5): the superposition
// phi = phi_P + V phi_L of the charge solution with the electrode at 0 V and
// the Laplace solution with it at 1 V (same operator), and the
// blocking-capacitor equation for the electrode potential V.
#include "ctx.h"

namespace rz {

namespace {

__device__ __forceinline__ double face_rule(double a, double b, int rule)
{
    return rule == 1 ? (a > b ? a : b) : 0.5 * (a + b);
}

__device__ __forceinline__ double block_sum256(double v, double *sh)
{
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0) sh[wv] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += sh[w];
    __syncthreads();
    return t;  // in thread 0
}

// Electrode charges of phi_P (with the deposited charge) and of phi_L, then
// the circuit update.  The charge of a potential u is Gauss's law on the
// union of the electrode nodes' half cells (0 <= z <= hz/2, r < R): the
// displacement eps0 (1 + chi) E leaving through their upper faces (area
// 2 pi r_j hr, pi hr^2 / 4 on the axis, at distance hz) and through the
// side face of the outermost one towards the wall node (area pi r hz at
// r = r_{nr-3/2}, distance hr), less the charge the deposit assigns to the
// half cells, rho V on row 0.  Charge arriving at the electrode since the
// previous solve comes from the z = 0 tallies of both species.  One block.
__global__ __launch_bounds__(256) void k_circuit(CircuitArgs a)
{
    __shared__ double sh[4];
    const int nr = a.nr;
    const double hr = a.hr, hz = a.hz;
    double qp = 0.0, ql = 0.0;
    for (int j = threadIdx.x; j < nr - 1; j += blockDim.x) {
        const double area = j == 0 ? kPi * 0.25 * hr * hr : 2.0 * kPi * (double)j * hr * hr;
        const double k = kEps0 * face_rule(a.eps[j], a.eps[nr + j], a.rule) * area / hz;
        qp += k * (a.phiP[j] - a.phiP[nr + j]) - a.rho[j] * a.vol[j];
        ql += k * (a.phiL[j] - a.phiL[nr + j]);
    }
    qp = block_sum256(qp, sh);
    ql = block_sum256(ql, sh);
    if (threadIdx.x != 0) return;
    const int jw = nr - 2;
    const double kw = kEps0 * face_rule(a.eps[jw], a.eps[jw + 1], a.rule) * kPi *
                      (((double)jw + 0.5) * hr) * hz / hr;
    qp += kw * (a.phiP[jw] - a.phiP[jw + 1]);
    ql += kw * (a.phiL[jw] - a.phiL[jw + 1]);
    CircuitState &s = *a.st;
    double qconv = 0.0;
    for (int sp = 0; sp < 2; ++sp) {
        const unsigned long long t = a.tally[3 * sp];
        qconv += a.q[sp] * ((double)(long long)(t - s.prev[sp]) * a.quantum[sp]);
        s.prev[sp] = t;
    }
    const double C = a.C, Vs = a.Vs;
    const double V = (s.Q - s.Qc + qconv + C * Vs - qp) / (ql + C);
    s.V = V;
    s.Q = qp + V * ql;
    s.Qc = C * (Vs - V);
    s.Qconv = qconv;
    s.Qp = qp;
    s.Ql = ql;
}

__global__ void k_combine(int nn, const double *phiP, const double *phiL, const CircuitState *st,
                          double *phi)
{
    const double V = st->V;
    for (int g = blockIdx.x * blockDim.x + threadIdx.x; g < nn; g += gridDim.x * blockDim.x)
        phi[g] = phiP[g] + V * phiL[g];
}

__global__ void k_circuit_set(CircuitState *st, double V, double Q, double Qc)
{
    st->V = V;
    st->Q = Q;
    st->Qc = Qc;
}

}  // namespace

hipError_t launch_circuit(const CircuitArgs &a, hipStream_t st)
{
    RZ_LAUNCH(k_circuit, dim3(1), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_combine(int nn, const double *phiP, const double *phiL, const CircuitState *cs,
                          double *phi, hipStream_t st)
{
    int threads = 256, blocks = (nn + threads - 1) / threads;
    RZ_LAUNCH(k_combine, dim3(blocks), dim3(threads), 0, st, nn, phiP, phiL, cs, phi);
    return hipGetLastError();
}

hipError_t launch_circuit_set(CircuitState *cs, double V, double Q, double Qc, hipStream_t st)
{
    RZ_LAUNCH(k_circuit_set, dim3(1), dim3(1), 0, st, cs, V, Q, Qc);
    return hipGetLastError();
}

}  // namespace rz
