// mc_thermo.hip -- the reduced reweighting of arXiv 0812.2964 (the paper's
// code (ii), Sec. 3.3, eq. reweighting2): the energy E, specific heat C, free
// energy F and entropy S of Sec. 4.1 at any inverse temperature, from the
// multicanonical weight alone.
//
// The density of states is inversely proportional to the weight, taken per
// reachable level m (E_m = 4m - 2N; levels 1 and N-1 do not exist) from the
// weight of its bin: ln D(m) = -ln w[m >> bs] + c, with c chosen so that D
// counts the 2^N configurations.  With p_m proportional to D(m) exp(-beta E_m):
//   E = sum p_m E_m,  C = beta^2 sum p_m (E_m - E)^2,
//   F = -ln Z / beta, S = beta (E - F),  ln Z = ln sum D(m) exp(-beta E_m),
// every sum taken in logarithms (shifted by its maximum) in binary64.
#include <mutex>

#include "mc_internal.h"

namespace mcgpu {

constexpr int kThermoThreads = 256;

// Sum (op 0) or maximum (op 1) over the workgroup, in a fixed order.
__device__ double block_reduce(double v, double *red, int op) {
    red[threadIdx.x] = v;
    __syncthreads();
    for (int h = kThermoThreads / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            const double o = red[threadIdx.x + h];
            red[threadIdx.x] = op == 0 ? red[threadIdx.x] + o : fmax(red[threadIdx.x], o);
        }
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}

// One workgroup per inverse temperature beta[k]; out[q * n_beta + k] for
// q = 0..3 = E, C, F, S.
__global__ __launch_bounds__(kThermoThreads) void k_thermo(SizeDev s, const double *beta_in, int n_beta,
                                                           double *out) {
    __shared__ double red[kThermoThreads];
    const int k = blockIdx.x;
    const int N = s.N;
    const double beta = beta_in[k];
    auto reachable = [&](int m) { return m != 1 && m != N - 1; };
    auto lnd = [&](int m) { return -s.lnW[m >> s.bin_shift]; };
    // normalisation: c = N ln 2 - ln sum_m exp(-ln w)
    double mx = -INFINITY;
    for (int m = threadIdx.x; m <= N; m += kThermoThreads)
        if (reachable(m)) mx = fmax(mx, lnd(m));
    mx = block_reduce(mx, red, 1);
    double sm = 0.0;
    for (int m = threadIdx.x; m <= N; m += kThermoThreads)
        if (reachable(m)) sm += exp(lnd(m) - mx);
    sm = block_reduce(sm, red, 0);
    const double c = (double)N * 0.69314718055994530942 - (mx + log(sm));
    // a_m = ln D(m) - beta E_m, without c (it cancels in E and C)
    auto a_of = [&](int m) { return lnd(m) - beta * (double)(4 * m - 2 * N); };
    double am = -INFINITY;
    for (int m = threadIdx.x; m <= N; m += kThermoThreads)
        if (reachable(m)) am = fmax(am, a_of(m));
    am = block_reduce(am, red, 1);
    double s0 = 0.0, s1 = 0.0;
    for (int m = threadIdx.x; m <= N; m += kThermoThreads) {
        if (!reachable(m)) continue;
        const double p = exp(a_of(m) - am);
        s0 += p;
        s1 += p * (double)(4 * m - 2 * N);
    }
    s0 = block_reduce(s0, red, 0);
    s1 = block_reduce(s1, red, 0);
    const double e_mean = s1 / s0;
    double s2 = 0.0;
    for (int m = threadIdx.x; m <= N; m += kThermoThreads) {
        if (!reachable(m)) continue;
        const double d = (double)(4 * m - 2 * N) - e_mean;
        s2 += exp(a_of(m) - am) * d * d;
    }
    s2 = block_reduce(s2, red, 0);
    if (threadIdx.x == 0) {
        const double lnZ = c + am + log(s0);
        const double f = -lnZ / beta;
        out[k] = e_mean;
        out[n_beta + k] = beta * beta * s2 / s0;
        out[2 * n_beta + k] = f;
        out[3 * n_beta + k] = beta * (e_mean - f);
    }
}

hipError_t launch_thermo(const SizeDev &s, const double *beta_dev, int n_beta, double *out_dev, hipStream_t st) {
    hipLaunchKernelGGL(k_thermo, dim3(n_beta), dim3(kThermoThreads), 0, st, s, beta_dev, n_beta, out_dev);
    return hipGetLastError();
}

// Device memory of mc_thermo_static: the inverse temperatures and the four
// results of at most kThermoStaticMaxBetas of them.  Every GPU the library
// runs on holds its own copy of the array until the process ends.
static __device__ __align__(256) double scratch[5 * kThermoStaticMaxBetas];

// In host code `scratch` names a host-side stand-in, not the device array, so
// its device address is looked up once per device, with that device current,
// and kept; callers use only the address returned here.
hipError_t thermo_scratch_address(int device, double **out) {
    static std::mutex mu;
    static double *addr[kMaxDevices] = {};
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        addr[device] = (double *)p;
    }
    *out = addr[device];
    return hipSuccess;
}

}  // namespace mcgpu
