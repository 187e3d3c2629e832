// Batched EM fit of one-dimensional Gaussian mixtures for gfx950: the pore-size
// distribution fit of arXiv:1601.00704, Sec. 2.2 (Eq. 20-24), for many sample
// sets at once (for instance one measured distribution per sample or region).
//
// One EM iteration is two launches.  k_gmm_pass walks a flat list of chunks of
// all active sets; every thread evaluates the responsibilities of Eq. (20) for
// its samples (log-sum-exp form, FP64) and accumulates, per component j,
//     S0 = sum w,  S1 = sum w (x - mu_j),  S2 = sum w (x - mu_j)^2
// (sums shifted by the current mean, so Eq. 24's variance is not formed as a
// difference of large squares) and the log-likelihood of the current
// parameters; a workgroup reduces them in a fixed order into its chunk's
// partial record.  k_gmm_update sums a set's chunk records in a fixed order
// (one workgroup per set) and applies Eq. (22)-(24):
//     Phi = S0 / m,  mu' = mu + S1 / S0,  var' = S2 / S0 - (S1 / S0)^2.
// Results are deterministic and independent of the batch composition.
// The kernel reads 8 bytes per sample and iteration and evaluates k
// exponentials (k - 1 for k = 2, whose larger term is 1) in FP64 per sample;
// the log-likelihood takes one logarithm per thread, of the product of its
// samples' sums (each in [1, k]).  It is bound by vector instruction issue,
// not by memory.
#include "glbm.h"
#include "glbm_internal.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <string>
#include <vector>

namespace {

constexpr int kGmmBlock = 256;
constexpr int kGmmPerThread = 16;
constexpr int kGmmChunk = kGmmBlock * kGmmPerThread;  // samples per chunk
constexpr int kGmmMaxK = GLBM_GMM_MAX_COMPONENTS;
constexpr int kRec = 3 * kGmmMaxK + 1;                 // S0, S1, S2 per component + log-likelihood
constexpr int kRecPad = 32;                            // doubles per chunk record

struct GmmSet {
    double phi[kGmmMaxK], mu[kGmmMaxK], var[kGmmMaxK];
    double la[kGmmMaxK];   // log(Phi_j / sqrt(2 pi var_j))
    double nb[kGmmMaxK];   // -1 / (2 var_j)
    double loglik, loglik_prev;
    int64_t off, n;        // samples [off, off + n) of the flat sample array
    int32_t chunk0, nchunk;
    int32_t active, iters;
};

struct GmmChunk {
    int32_t set;
    int32_t pad;
    int64_t start;   // first sample of the chunk (absolute index)
    int64_t end;     // one past the last
};

__device__ __forceinline__ void prepare(GmmSet& S, int k)
{
    for (int j = 0; j < k; ++j) {
        S.la[j] = log(S.phi[j]) - 0.5 * log(2.0 * 3.14159265358979323846 * S.var[j]);
        S.nb[j] = -0.5 / S.var[j];
    }
}

__global__ void k_gmm_prepare(GmmSet* sets, int n_sets, int k)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s < n_sets) prepare(sets[s], k);
}

// ln 2 split for the range reductions below: kLn2Hi holds its leading 32
// bits (so k kLn2Hi is exact for |k| < 2^21), kLn2Lo the rest.
constexpr double kLn2Hi = 0x1.62e42ffp-1;
constexpr double kLn2Lo = -4.2009150726810846e-11;

// Series coefficients, passed to the pass as a kernel argument so that they sit
// in scalar registers (a literal coefficient is rebuilt in a vector register at
// every use): 1/13!, 1/12!, ..., 1/2!, 1, 1, the Taylor series of e^r, highest
// degree first.
struct GmmSeries {
    double exp_c[14];
};

GmmSeries gmm_series()
{
    GmmSeries c;
    double f = 1.0;
    for (int n = 1; n <= 13; ++n) f *= n;  // 13!, exact in double
    for (int n = 13; n >= 0; --n) {
        c.exp_c[13 - n] = 1.0 / f;
        if (n > 0) f /= n;
    }
    return c;
}

// 1/y for y in [1, 4]: the hardware reciprocal estimate refined by two Newton
// steps, e = 1 - y r, r <- r + r e (each step squares the relative error).  In
// that range no operand scaling or special case arises, so the scaling and
// fix-up steps of a full division are not needed; the result is within about
// one unit in the last place, where a division would be correctly rounded.
__device__ __forceinline__ double rcp_1_4(double y)
{
    double r = __builtin_amdgcn_rcp(y);
    double e = fma(-y, r, 1.0);
    r = fma(r, e, r);
    e = fma(-y, r, 1.0);
    return fma(r, e, r);
}

// e^a for a <= 0, written from the mathematics: a = k ln 2 + r with
// |r| <= ln 2 / 2, e^r by its Taylor series to degree 13 (truncation below
// 5e-18 relative on that interval, Horner form), then the exact scaling by
// 2^k.  Below -745 the result is 0 (it would be a denormal or zero anyway).
__device__ __forceinline__ double exp_nonpos(double a, const GmmSeries& C)
{
    if (a < -745.0) return 0.0;
    const double k = rint(a * 1.4426950408889634);
    const double r = fma(-k, kLn2Lo, fma(-k, kLn2Hi, a));
    double p = C.exp_c[0];
#pragma unroll
    for (int c = 1; c < 14; ++c) p = fma(p, r, C.exp_c[c]);
    return ldexp(p, (int)k);
}

template <int K>
__global__ __launch_bounds__(kGmmBlock) void k_gmm_pass(const double* __restrict__ x, const GmmSet* __restrict__ sets,
                                                          const GmmChunk* __restrict__ chunks, double* __restrict__ part,
                                                          GmmSeries ser)
{
    __shared__ double red[kGmmBlock / 64][kRec];
    const GmmChunk c = chunks[blockIdx.x];
    const GmmSet& S = sets[c.set];
    if (!S.active) return;
    double mu[K], la[K], nb[K];
#pragma unroll
    for (int j = 0; j < K; ++j) {
        mu[j] = S.mu[j];
        la[j] = S.la[j];
        nb[j] = S.nb[j];
    }
    double acc[3 * K + 1];
#pragma unroll
    for (int r = 0; r < 3 * K + 1; ++r) acc[r] = 0.0;
    // log-likelihood: sum of the per-sample maxima, plus one logarithm of the
    // product of the per-sample sums (at most kGmmPerThread factors in [1, K])
    static_assert(kGmmPerThread <= 16 && kGmmMaxK <= 8, "the product of the sums must stay below 2^48");
    double prod = 1.0;
    // the next sample is loaded before the current one is evaluated
    int64_t i = c.start + threadIdx.x;
    double xn = i < c.end ? x[i] : 0.0;
    for (; i < c.end; i += kGmmBlock) {
        const double xi = xn;
        if (i + kGmmBlock < c.end) xn = x[i + kGmmBlock];
        double t[K], d[K];
#pragma unroll
        for (int j = 0; j < K; ++j) {
            d[j] = xi - mu[j];
            t[j] = la[j] + nb[j] * d[j] * d[j];   // log(Phi_j g_j(x)), Eq. (21)
        }
        double w[K], mx;                          // responsibilities of Eq. (20), larger term
        if constexpr (K == 2) {
            // the larger term is exp(0) = 1: one exponential, and the sum lies in [1, 2]
            const bool first = t[0] >= t[1];
            mx = first ? t[0] : t[1];
            const double o = exp_nonpos(-fabs(t[1] - t[0]), ser);
            const double sum = 1.0 + o;
            prod *= sum;
            const double inv = rcp_1_4(sum), wo = o * inv;
            w[0] = first ? inv : wo;
            w[1] = first ? wo : inv;
        } else {
            mx = -INFINITY;
#pragma unroll
            for (int j = 0; j < K; ++j) mx = fmax(mx, t[j]);
            double e[K], sum = 0.0;
#pragma unroll
            for (int j = 0; j < K; ++j) {
                e[j] = exp(t[j] - mx);
                sum += e[j];
            }
            prod *= sum;
            const double inv = 1.0 / sum;
#pragma unroll
            for (int j = 0; j < K; ++j) w[j] = e[j] * inv;
        }
#pragma unroll
        for (int j = 0; j < K; ++j) {
            acc[3 * j] += w[j];
            acc[3 * j + 1] += w[j] * d[j];
            acc[3 * j + 2] += w[j] * d[j] * d[j];
        }
        acc[3 * K] += mx;
    }
    acc[3 * K] += log(prod);
    // wavefront trees, then the four wavefronts in a fixed order
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
    for (int r = 0; r < 3 * K + 1; ++r) {
        double v = acc[r];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
        if (lane == 0) red[wave][r] = v;
    }
    __syncthreads();
    if (threadIdx.x < 3 * K + 1) {
        const int r = threadIdx.x;
        double v = red[0][r];
        for (int w = 1; w < kGmmBlock / 64; ++w) v += red[w][r];
        part[(size_t)blockIdx.x * kRecPad + r] = v;
    }
}

// One workgroup per set: fixed-order sum of the chunk records, then Eq. (22)-(24).
// with_update = 0: only the log-likelihood of the current parameters.
__global__ __launch_bounds__(kGmmBlock) void k_gmm_update(GmmSet* sets, const double* __restrict__ part, int k,
                                                            double tol, int with_update)
{
    __shared__ double red[kGmmBlock];
    GmmSet& S = sets[blockIdx.x];
    if (!S.active) return;
    const int nrec = 3 * k + 1;
    // thread t keeps record component t % kRecPad of chunks t / kRecPad, + 8, ...
    const int comp = threadIdx.x % kRecPad, c0 = threadIdx.x / kRecPad;
    constexpr int kStep = kGmmBlock / kRecPad;
    double acc = 0.0;
    if (comp < nrec) {
        // eight loads in flight, added in chunk order (the same sum as one at a time)
        const double* __restrict__ p = part + (size_t)S.chunk0 * kRecPad + comp;
        int ch = c0;
        for (; ch + 7 * kStep < S.nchunk; ch += 8 * kStep) {
            double v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = p[(size_t)(ch + u * kStep) * kRecPad];
#pragma unroll
            for (int u = 0; u < 8; ++u) acc += v[u];
        }
        for (; ch < S.nchunk; ch += kStep) acc += p[(size_t)ch * kRecPad];
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = kGmmBlock / 2; w >= kRecPad; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    const double L = red[3 * k];
    S.loglik_prev = S.loglik;
    S.loglik = L;
    if (!with_update) return;
    for (int j = 0; j < k; ++j) {
        const double s0 = red[3 * j], s1 = red[3 * j + 1], s2 = red[3 * j + 2];
        if (!(s0 > 0.0)) {
            // an empty component: Eq. (22) gives Phi = 0; Eq. (23)-(24) are 0/0,
            // so its mean and variance are kept
            if (s0 == 0.0) S.phi[j] = 0.0;
            continue;
        }
        const double dm = s1 / s0;
        S.phi[j] = s0 / (double)S.n;          // Eq. (22)
        S.mu[j] += dm;                        // Eq. (23)
        S.var[j] = s2 / s0 - dm * dm;         // Eq. (24), about the updated mean
    }
    prepare(S, k);
    S.iters += 1;
    // stop after an iteration whose log-likelihood gain (of the parameters it
    // started from over the previous ones) is within tol of the log-likelihood
    if (tol > 0.0 && S.iters >= 2 && S.loglik - S.loglik_prev <= tol * fabs(S.loglik)) S.active = 0;
}

thread_local std::string g_gmm_err;
int gfail(int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    glbm::set_error(buf);
    return code;
}

#define GCHK(expr)                                                                                     \
    do {                                                                                               \
        hipError_t e_ = (expr);                                                                        \
        if (e_ != hipSuccess) return gfail(GLBM_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_));       \
    } while (0)

template <int K> hipError_t launch_pass(int nchunks, const double* x, const GmmSet* sets, const GmmChunk* ch,
                                        double* part, hipStream_t s)
{
    hipLaunchKernelGGL(k_gmm_pass<K>, dim3(nchunks), dim3(kGmmBlock), 0, s, x, sets, ch, part, gmm_series());
    return hipGetLastError();
}

hipError_t pass(int k, int nchunks, const double* x, const GmmSet* sets, const GmmChunk* ch, double* part,
                hipStream_t s)
{
    switch (k) {
    case 1: return launch_pass<1>(nchunks, x, sets, ch, part, s);
    case 2: return launch_pass<2>(nchunks, x, sets, ch, part, s);
    case 3: return launch_pass<3>(nchunks, x, sets, ch, part, s);
    case 4: return launch_pass<4>(nchunks, x, sets, ch, part, s);
    case 5: return launch_pass<5>(nchunks, x, sets, ch, part, s);
    case 6: return launch_pass<6>(nchunks, x, sets, ch, part, s);
    case 7: return launch_pass<7>(nchunks, x, sets, ch, part, s);
    case 8: return launch_pass<8>(nchunks, x, sets, ch, part, s);
    default: return hipErrorInvalidValue;
    }
}

// Device buffers of one fit, freed on every exit path.
struct GmmBuffers {
    GmmSet* sets = nullptr;
    GmmChunk* chunks = nullptr;
    double* part = nullptr;
    ~GmmBuffers()
    {
        if (sets) (void)hipFree(sets);
        if (chunks) (void)hipFree(chunks);
        if (part) (void)hipFree(part);
    }
};

}  // namespace

extern "C" int glbm_gmm_fit(int32_t n_sets, const int64_t* offsets, const double* x_dev, int32_t k, double* phi,
                            double* mu, double* var, int32_t iters, double tol, double* loglik, int32_t* iters_done,
                            void* hip_stream)
{
    glbm::set_error("");
    if (n_sets < 1 || !offsets || !x_dev || !phi || !mu || !var) return gfail(GLBM_EINVAL, "null or empty argument");
    if (k < 1 || k > kGmmMaxK) return gfail(GLBM_EINVAL, "k must be in [1, %d]", kGmmMaxK);
    if (iters < 0) return gfail(GLBM_EINVAL, "iters must be >= 0");
    if (!(tol >= 0.0) || !std::isfinite(tol)) return gfail(GLBM_EINVAL, "tol must be finite and >= 0");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    std::vector<GmmSet> sh(n_sets);
    std::vector<GmmChunk> ch;
    for (int i = 0; i < n_sets; ++i) {
        const int64_t a = offsets[i], b = offsets[i + 1];
        if (a < 0 || b <= a) return gfail(GLBM_EINVAL, "set %d: empty or decreasing sample range", i);
        GmmSet& S = sh[i];
        S = GmmSet{};
        double fsum = 0.0;
        for (int j = 0; j < k; ++j) {
            const double p = phi[i * k + j], m = mu[i * k + j], v = var[i * k + j];
            if (!(p > 0.0) || !(v > 0.0) || !std::isfinite(p) || !std::isfinite(m) || !std::isfinite(v))
                return gfail(GLBM_EINVAL, "set %d component %d: need Phi > 0, var > 0, all finite", i, j);
            S.phi[j] = p;
            S.mu[j] = m;
            S.var[j] = v;
            fsum += p;
        }
        if (std::fabs(fsum - 1.0) > 1e-9) return gfail(GLBM_EINVAL, "set %d: fractions sum to %g, not 1", i, fsum);
        S.off = a;
        S.n = b - a;
        S.chunk0 = (int32_t)ch.size();
        for (int64_t c = a; c < b; c += kGmmChunk) ch.push_back(GmmChunk{i, 0, c, std::min<int64_t>(c + kGmmChunk, b)});
        S.nchunk = (int32_t)ch.size() - S.chunk0;
        S.active = 1;
        S.iters = 0;
        S.loglik = S.loglik_prev = -INFINITY;
    }
    if (ch.size() > (size_t)INT32_MAX) return gfail(GLBM_EINVAL, "too many samples");
    GmmBuffers B;
    GCHK(hipMalloc(&B.sets, sh.size() * sizeof(GmmSet)));
    GCHK(hipMalloc(&B.chunks, ch.size() * sizeof(GmmChunk)));
    GCHK(hipMalloc(&B.part, ch.size() * kRecPad * sizeof(double)));
    GCHK(hipMemcpyAsync(B.sets, sh.data(), sh.size() * sizeof(GmmSet), hipMemcpyHostToDevice, s));
    GCHK(hipMemcpyAsync(B.chunks, ch.data(), ch.size() * sizeof(GmmChunk), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_gmm_prepare, dim3((n_sets + 255) / 256), dim3(256), 0, s, B.sets, n_sets, k);
    GCHK(hipGetLastError());
    const int nch = (int)ch.size();
    for (int it = 0; it < iters; ++it) {
        GCHK(pass(k, nch, x_dev, B.sets, B.chunks, B.part, s));
        hipLaunchKernelGGL(k_gmm_update, dim3(n_sets), dim3(kGmmBlock), 0, s, B.sets, B.part, k, tol, 1);
        GCHK(hipGetLastError());
        if (tol > 0.0 && (it % 16) == 15) {
            // stop early once every set has converged
            GCHK(hipMemcpyAsync(sh.data(), B.sets, sh.size() * sizeof(GmmSet), hipMemcpyDeviceToHost, s));
            GCHK(hipStreamSynchronize(s));
            bool any = false;
            for (const auto& S : sh) any |= S.active != 0;
            if (!any) break;
        }
    }
    // log-likelihood of the returned parameters: one E pass without an update, every set
    GCHK(hipMemcpyAsync(sh.data(), B.sets, sh.size() * sizeof(GmmSet), hipMemcpyDeviceToHost, s));
    GCHK(hipStreamSynchronize(s));
    std::vector<int32_t> iters_of(n_sets);
    for (int i = 0; i < n_sets; ++i) {
        iters_of[i] = sh[i].iters;
        sh[i].active = 1;
    }
    GCHK(hipMemcpyAsync(B.sets, sh.data(), sh.size() * sizeof(GmmSet), hipMemcpyHostToDevice, s));
    GCHK(pass(k, nch, x_dev, B.sets, B.chunks, B.part, s));
    hipLaunchKernelGGL(k_gmm_update, dim3(n_sets), dim3(kGmmBlock), 0, s, B.sets, B.part, k, 0.0, 0);
    GCHK(hipGetLastError());
    GCHK(hipMemcpyAsync(sh.data(), B.sets, sh.size() * sizeof(GmmSet), hipMemcpyDeviceToHost, s));
    GCHK(hipStreamSynchronize(s));
    for (int i = 0; i < n_sets; ++i) {
        for (int j = 0; j < k; ++j) {
            phi[i * k + j] = sh[i].phi[j];
            mu[i * k + j] = sh[i].mu[j];
            var[i * k + j] = sh[i].var[j];
        }
        if (loglik) loglik[i] = sh[i].loglik;
        if (iters_done) iters_done[i] = iters_of[i];
    }
    return GLBM_OK;
}
