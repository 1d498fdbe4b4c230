// A-posteriori error quantities of Section 3.1: eta = d_min / ||W||_inf of the
// Lemma on normalisation, the sampled kernel error ||K_ERR||_inf of
// eq. KERR_estimate and the estimate eps <~ n ||K_ERR||_inf / ||W||_inf of
// eq. epsilon_KERR_estimate.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <limits>
#include <vector>

#include "nfl_internal.h"

namespace nfl {

constexpr int KE_THREADS = 256;

// diff[s] = |kr[s] - K_RF(y_s)| with K_RF(y) = sum_{l in I_N^d} b_l cos(2 pi l.y)
// (the real part of eq. K_RF; b_l is real).  One workgroup per sample point;
// the phases e^{2 pi i l_t y_t} of each axis sit in LDS, the terms are summed
// per thread in index order and then over the workgroup in a fixed tree.
__global__ __launch_bounds__(KE_THREADS) void k_kerr(const double *__restrict__ bhat, int d, int N,
                                                     const double *__restrict__ y,
                                                     const double *__restrict__ kr,
                                                     double *__restrict__ diff) {
  extern __shared__ double2 ph[];   // d x N, axis t at t*N + (l mod N)
  __shared__ double red[KE_THREADS / 64];
  const int s = blockIdx.x;
  for (int k = threadIdx.x; k < d * N; k += KE_THREADS) {
    const int t = k / N, lm = k - t * N;
    const int l = lm < N / 2 ? lm : lm - N;
    double sn, cs;
    sincospi(2.0 * (double)l * y[(size_t)s * d + t], &sn, &cs);
    ph[k] = make_double2(cs, sn);
  }
  __syncthreads();
  size_t tot = 1;
  for (int t = 0; t < d; ++t) tot *= (size_t)N;
  double acc = 0.0;
  for (size_t q = threadIdx.x; q < tot; q += KE_THREADS) {
    size_t r = q;
    double2 e = make_double2(1.0, 0.0);
    for (int t = d - 1; t >= 0; --t) {
      const double2 f = ph[t * N + (int)(r % (size_t)N)];
      r /= (size_t)N;
      e = make_double2(e.x * f.x - e.y * f.y, e.x * f.y + e.y * f.x);
    }
    acc += bhat[q] * e.x;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double sum = 0.0;
    for (int w = 0; w < KE_THREADS / 64; ++w) sum += red[w];
    diff[s] = fabs(kr[s] - sum);
  }
}

static uint64_t splitmix_next(uint64_t &st) {
  uint64_t z = (st += 0x9e3779b97f4a7c15ULL);
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
  return z ^ (z >> 31);
}

static double uniform01(uint64_t &st) {   // in (0, 1)
  return ((splitmix_next(st) >> 11) + 0.5) * (1.0 / 9007199254740992.0);
}

// S points uniform in the ball ||y|| <= R of R^d: a direction from d normal
// deviates (Box-Muller), a radius R u^{1/d}.
static void ball_samples(int S, int d, double R, uint64_t seed, std::vector<double> &y) {
  uint64_t st = seed * 0x2545f4914f6cdd1dULL + 0x632be59bd9b4e019ULL;
  y.assign((size_t)S * d, 0.0);
  for (int s = 0; s < S; ++s) {
    double g[3], nrm = 0.0;
    do {
      nrm = 0.0;
      for (int t = 0; t < d; ++t) {
        const double u1 = uniform01(st), u2 = uniform01(st);
        g[t] = std::sqrt(-2.0 * std::log(u1)) * std::cos(2.0 * M_PI * u2);
        nrm += g[t] * g[t];
      }
    } while (nrm == 0.0);
    const double r = R * std::pow(uniform01(st), 1.0 / d) / std::sqrt(nrm);
    for (int t = 0; t < d; ++t) y[(size_t)s * d + t] = g[t] * r;
  }
}

int error_estimate(nfl_plan *P, int S, uint64_t seed, const double *y_host, double *eta,
                   double *kerr, double *eps_est, double *bound) {
  const int d = P->d, N = P->N;
  const RegKernel KR(P->kind, P->sigma_t, P->eps_B, P->eps_I, P->p);
  std::vector<double> bhat, y, kr((size_t)S);
  kernel_bhat(d, N, KR, bhat);
  if (y_host) {
    y.assign(y_host, y_host + (size_t)S * d);
  } else {
    ball_samples(S, d, 0.5 - P->eps_B, seed, y);
  }
  for (int s = 0; s < S; ++s) {
    double rr = 0.0;
    for (int t = 0; t < d; ++t) rr += y[(size_t)s * d + t] * y[(size_t)s * d + t];
    kr[s] = KR(std::sqrt(rr));
  }
  LBuf<double> bd, yd, krd, df;
  NFL_TRY(bd.ensure(bhat.size()));
  NFL_TRY(yd.ensure(y.size()));
  NFL_TRY(krd.ensure(kr.size()));
  NFL_TRY(df.ensure((size_t)S));
  hipStream_t st = P->stream;
  NFL_HIP(hipMemcpyAsync(bd.p, bhat.data(), bhat.size() * sizeof(double), hipMemcpyHostToDevice, st));
  NFL_HIP(hipMemcpyAsync(yd.p, y.data(), y.size() * sizeof(double), hipMemcpyHostToDevice, st));
  NFL_HIP(hipMemcpyAsync(krd.p, kr.data(), kr.size() * sizeof(double), hipMemcpyHostToDevice, st));
  hipLaunchKernelGGL(k_kerr, dim3(S), dim3(KE_THREADS), (size_t)d * N * sizeof(double2), st, bd.p,
                     d, N, yd.p, krd.p, df.p);
  NFL_HIP(hipGetLastError());
  std::vector<double> diff((size_t)S);
  NFL_HIP(hipMemcpyAsync(diff.data(), df.p, diff.size() * sizeof(double), hipMemcpyDeviceToHost, st));
  NFL_HIP(hipStreamSynchronize(st));
  const double ke = *std::max_element(diff.begin(), diff.end());
  // the kernels here are positive, so ||W||_inf is the largest degree; the
  // plan's degrees are the approximate ones, d_E (the only ones it has)
  const double winf = P->dmax, et = P->dmin / P->dmax;
  const double ep = (double)P->n * ke / winf;
  if (eta) *eta = et;
  if (kerr) *kerr = ke;
  if (eps_est) *eps_est = ep;
  if (bound)
    *bound = ep < et ? ep * (1.0 + et) / (et * (et - ep)) : std::numeric_limits<double>::infinity();
  return NFL_OK;
}

}  // namespace nfl

using namespace nfl;

extern "C" int nfl_error_estimate(nfl_handle P, int nsamples, uint64_t seed, const double *y_host,
                                  double *eta, double *kerr_inf, double *eps_est,
                                  double *lemma_bound) {
  if (!P) { set_error("null handle"); return NFL_ERR_ARG; }
  if (!P->have_kernel) { set_error("error estimate before a successful nfl_set_kernel"); return NFL_ERR_ORDER; }
  if (P->frame_only) { set_error("error estimate on a plan of target nodes: it has no degrees"); return NFL_ERR_ORDER; }
  if (nsamples < 1 || nsamples > (1 << 20)) { set_error("need 1 <= nsamples <= 2^20"); return NFL_ERR_ARG; }
  if (y_host) {
    const double R = 0.5 - P->eps_B;
    for (int64_t k = 0; k < (int64_t)nsamples; ++k) {
      double rr = 0.0;
      for (int t = 0; t < P->d; ++t) rr += y_host[k * P->d + t] * y_host[k * P->d + t];
      if (!(rr <= R * R * (1.0 + 1e-12))) { set_error("sample point outside the ball ||y|| <= 1/2 - eps_B"); return NFL_ERR_ARG; }
    }
  }
  return error_estimate(P, nsamples, seed, y_host, eta, kerr_inf, eps_est, lemma_bound);
}
