// Diagnostic reductions over moment fields: the domain averages of the
// moment magnitudes that Sec. III.B plots (<|n_ab|>, <|f^(x)_ab|> for
// neutrinos and antineutrinos).  Deterministic two-level sums: block b sums
// cells b*256 + t, b*256 + t + nblk*256, ... per thread, a fixed LDS tree per
// block, then the blocks in order.
#include "fpic_diag.h"

namespace fpic {

namespace {

constexpr int NQ = 24;  // 4 fields x (3 diagonal + 3 off-diagonal)

__global__ void __launch_bounds__(256)
domain_sums_kernel(const double *__restrict__ m, int64_t nc, double *__restrict__ partial)
{
    __shared__ double sh[256];
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int q = 0; q < NQ; ++q) {
        // field: n (row 0), f_x (9), nbar (36), fbar_x (45); packed entry
        const int f = q / 6, e = q % 6;
        const int base = (f == 0) ? 0 : (f == 1) ? 9 : (f == 2) ? 36 : 45;
        double s = 0.0;
        for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < nc; c += stride) {
            if (e < 3) {
                s += fabs(m[(base + e) * nc + c]);
            } else {
                const int k = base + 3 + 2 * (e - 3);
                s += hypot(m[k * nc + c], m[(k + 1) * nc + c]);
            }
        }
        sh[threadIdx.x] = s;
        __syncthreads();
        for (int h = 128; h > 0; h >>= 1) {
            if ((int)threadIdx.x < h)
                sh[threadIdx.x] += sh[threadIdx.x + h];
            __syncthreads();
        }
        if (threadIdx.x == 0)
            partial[(size_t)blockIdx.x * NQ + q] = sh[0];
        __syncthreads();
    }
}

__global__ void domain_sums_finish(const double *__restrict__ partial, int nblk, double *__restrict__ out)
{
    const int q = threadIdx.x;
    if (q >= NQ)
        return;
    double s = 0.0;
    for (int b = 0; b < nblk; ++b)
        s += partial[(size_t)b * NQ + q];
    out[q] = s;
}

}  // namespace

hipError_t launch_domain_sums(const double *m, int64_t ncell, int nblk, double *scratch,
                              double *out24, hipStream_t s)
{
    domain_sums_kernel<<<nblk, 256, 0, s>>>(m, ncell, scratch);
    domain_sums_finish<<<1, 64, 0, s>>>(scratch, nblk, out24);
    return hipGetLastError();
}

}  // namespace fpic
