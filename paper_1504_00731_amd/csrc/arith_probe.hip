// Probes of the kernels' device arithmetic: the division, reciprocal, square
// root and WENO-theta routines the sweep kernels use, applied elementwise to
// arrays, so that GPU tests can compare them with IEEE results and with the
// oracle over many inputs.  Built as its own library (libwt_probe.so); not
// part of the solver's interface.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "wt_round.hpp"
#include "wt_weno.hpp"

namespace {

constexpr int kProbeThreads = 256;

enum ProbeOp : int {
    kDiv = 0,            // out = a / b                      (a, b: n values)
    kRecip = 1,          // out = 1 / b                      (b: n values)
    kDivByRecip = 2,     // out = a / c0 from c1 = RN(1/c0)  (a: n values)
    kSqrt = 3,           // out = sqrt(a)                    (a: n values)
    kWeno = 4,           // FP64 WENO-theta, eps c0, alpha_R c1, RN(1/eps) c2 (a: 6 n values)
    kWenoFp32 = 5,       // FP32 reconstruction, eps c0, alpha_R c1 (a: 6 n values)
    kRcpFast = 6,        // out = 1 / b, the fast modes' reciprocal (b: n values)
    kRcpEstimate = 7,    // out = the hardware reciprocal estimate of b (b: n values)
    kWenoFast = 8,       // fast FP64 WENO-theta, eps c0, alpha_R c1 (a: 6 n values)
    kRsqFast = 9,        // out = 1 / sqrt(b), the fast modes' reciprocal square root (b: n values)
    kSqrtFast = 10,      // out = sqrt(b), the fast modes' square root (b: n values)
};

__global__ __launch_bounds__(kProbeThreads) void probe_kernel(int op, const double *a,
                                                              const double *b, double c0,
                                                              double c1, double c2, double *out,
                                                              int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * kProbeThreads + threadIdx.x;
    if (i >= n) return;
    switch (op) {
    case kDiv: out[i] = wt::div_rn(a[i], b[i]); break;
    case kRecip: out[i] = wt::recip_rn(b[i]); break;
    case kDivByRecip: out[i] = wt::div_by_recip_checked(a[i], c0, c1); break;
    case kSqrt: out[i] = wt::sqrt_rn(a[i]); break;
    case kWeno: {
        const double *s = a + 6 * i;
        out[i] = wt::weno_theta(s[0], s[1], s[2], s[3], s[4], s[5], c0, c1, c2);
        break;
    }
    case kWenoFp32: out[i] = wt::weno_theta_fp32_recon(a + 6 * i, c0, (float)c1); break;
    case kRcpFast: out[i] = wt::rcp_fast(b[i]); break;
    case kRcpEstimate: out[i] = __builtin_amdgcn_rcp(b[i]); break;
    case kWenoFast: {
        const double *s = a + 6 * i;
        out[i] = wt::weno_theta_fast(s[0], s[1], s[2], s[3], s[4], s[5], c0, c1);
        break;
    }
    case kRsqFast: out[i] = wt::rsq_fast(b[i]); break;
    case kSqrtFast: out[i] = wt::sqrt_fast(b[i]); break;
    default: break;
    }
}

}  // namespace

// Applies probe `op` to n elements on `stream` (device pointers; a holds 6 n
// values for the WENO probes, n otherwise; b is read by kDiv, the reciprocals and
// the fast roots, which do not read a).
// Returns 0, 1 for bad arguments, 5 if the launch failed.  Asynchronous.
extern "C" int wt_probe(int op, const double *a, const double *b, double c0, double c1, double c2,
                        double *out, int64_t n, void *stream)
{
    if (op < kDiv || op > kSqrtFast || n < 0 || !out) return 1;
    const bool b_only = op == kRecip || op == kRcpFast || op == kRcpEstimate || op == kRsqFast ||
                        op == kSqrtFast;
    if ((b_only || op == kDiv) && !b) return 1;
    if (!b_only && !a) return 1;
    if (n == 0) return 0;
    const int64_t blocks = (n + kProbeThreads - 1) / kProbeThreads;
    if (blocks > 0x7fffffff) return 1;
    hipLaunchKernelGGL(probe_kernel, dim3((unsigned)blocks), dim3(kProbeThreads), 0,
                       (hipStream_t)stream, op, a, b, c0, c1, c2, out, n);
    return hipGetLastError() == hipSuccess ? 0 : 5;
}
