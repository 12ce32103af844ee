// qmc_noalloc.hip -- qmc_observe_noalloc: the estimators of qmc_observe (eq. (3) numerators,
// trace, sign angle, Pauli expectations, fidelity, anti-Hermiticity) on a sorted store that the
// caller holds in device memory, for callers that cannot allocate.  No context, no device or host
// allocation: every scratch word (inputs staged on the device, per-replica accumulators, lookups,
// replica bounds, outputs in the caller's layouts) lives in one file-scope device array, whose
// address is taken once per device with hipGetSymbolAddress.  The estimator passes are the
// kernels of qmc_observe (k_observe, k_lookup); the set-up and the FP64 normalization are kernels
// of this file.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <mutex>

#include "../../include/qmc.h"
#include "qmc_device.hpp"
#include "qmc_kernels.h"

namespace {

using qmc::kBlock;

constexpr uint32_t kNaReplicas = QMC_NOALLOC_MAX_REPLICAS;
constexpr uint32_t kNaPauli = QMC_NOALLOC_MAX_PAULI;
constexpr uint32_t kNaPsi = QMC_NOALLOC_MAX_PSI;
constexpr uint32_t kNaLookTotal = QMC_NOALLOC_MAX_LOOKUPS;
constexpr uint32_t kNaStride = 5 + 2 * kNaPauli;  // accumulator words per replica (k_observe)

constexpr size_t al(size_t v) { return (v + 255) & ~size_t(255); }

// Parts of the scratch array, in bytes from its start.
constexpr size_t kOffCnt = 0;  // Counters image: n_store[0] = the store size
constexpr size_t kOffPx = kOffCnt + al(sizeof(qmc::Counters));
constexpr size_t kOffPz = kOffPx + al(8 * kNaPauli);
constexpr size_t kOffPxz = kOffPz + al(8 * kNaPauli);
constexpr size_t kOffPidx = kOffPxz + al(16 * kNaPauli);
constexpr size_t kOffPre = kOffPidx + al(8 * kNaPsi);
constexpr size_t kOffPim = kOffPre + al(8 * kNaPsi);
constexpr size_t kOffLook = kOffPim + al(8 * kNaPsi);
constexpr size_t kOffNd0 = kOffLook + al(8 * kNaPsi * kNaPsi);
constexpr size_t kOffAcc = kOffNd0 + al(8 * kNaReplicas);
constexpr size_t kOffLout = kOffAcc + al(8 * (size_t)kNaReplicas * kNaStride);
constexpr size_t kOffBnd = kOffLout + al(16 * (size_t)kNaLookTotal);
constexpr size_t kOffOcc = kOffBnd + al(8 * (kNaReplicas + 1));
constexpr size_t kOffTot = kOffOcc + al(8 * kNaReplicas);
constexpr size_t kOffNdg = kOffTot + al(8 * kNaReplicas);
constexpr size_t kOffPau = kOffNdg + al(16 * kNaReplicas);
constexpr size_t kOffEps2 = kOffPau + al(16 * (size_t)kNaReplicas * kNaPauli);
constexpr size_t kOffTr = kOffEps2 + al(16 * kNaReplicas);
constexpr size_t kOffTh = kOffTr + al(8 * kNaReplicas);
constexpr size_t kOffPv = kOffTh + al(8 * kNaReplicas);
constexpr size_t kOffFid = kOffPv + al(16 * (size_t)kNaReplicas * kNaPauli);
constexpr size_t kOffEps = kOffFid + al(16 * kNaReplicas);
constexpr size_t kScratchBytes = kOffEps + al(8 * kNaReplicas);
static_assert(kScratchBytes == QMC_NOALLOC_SCRATCH_BYTES,
              "qmc.h states the scratch size of qmc_observe_noalloc");

// The scratch of qmc_observe_noalloc.  In host code this name is not a device address: host code
// uses the per-device pointer that hipGetSymbolAddress returns (scratch_of_current_device).
static __device__ __align__(256) uint8_t scratch[kScratchBytes];

constexpr int kNaDevices = 64;
std::mutex g_mu;
uint8_t* g_ptr[kNaDevices];  // the scratch address on each device, once taken

// The scratch address on the current device, taken once per device.
hipError_t scratch_of_current_device(uint8_t** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kNaDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_ptr[dev] = static_cast<uint8_t*>(p);
  }
  *out = g_ptr[dev];
  return hipSuccess;
}

template <class T>
__host__ __device__ T* part(uint8_t* base, size_t off) {
  return reinterpret_cast<T*>(base + off);
}

// Store size into the Counters image, accumulators cleared, Pauli masks interleaved as k_observe
// reads them, and the lookup keys (bra psi_v, ket psi_u) in the order qmc_observe uses.
__global__ void k_na_prepare(uint8_t* __restrict__ sc, uint64_t n, uint32_t nacc, uint32_t npl,
                             uint32_t npsi, uint32_t nq) {
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x, T = gridDim.x * blockDim.x;
  if (t == 0) part<qmc::Counters>(sc, kOffCnt)->n_store[0] = n;
  unsigned long long* acc = part<unsigned long long>(sc, kOffAcc);
  for (uint32_t i = t; i < nacc; i += T) acc[i] = 0;
  const uint64_t* px = part<uint64_t>(sc, kOffPx);
  const uint64_t* pz = part<uint64_t>(sc, kOffPz);
  uint64_t* pxz = part<uint64_t>(sc, kOffPxz);
  for (uint32_t k = t; k < npl; k += T) {
    pxz[2 * k] = px[k];
    pxz[2 * k + 1] = pz[k];
  }
  const uint64_t* pidx = part<uint64_t>(sc, kOffPidx);
  uint64_t* lk = part<uint64_t>(sc, kOffLook);
  for (uint32_t i = t; i < npsi * npsi; i += T) {
    const uint32_t u = i / npsi, v = i % npsi;
    lk[i] = (pidx[v] << nq) | pidx[u];
  }
}

// Per-replica outputs from the accumulators, the lookups and the replica bounds, in the layouts
// of qmc_obs_out, with the operations of qmc_observe in the same order (one thread per replica).
__global__ void k_na_finish(uint8_t* __restrict__ sc, uint32_t R, uint32_t npl, uint32_t npsi) {
  const uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= R) return;
  const uint32_t stride = 5 + 2 * npl, nlook = npsi * npsi;
  const unsigned long long* a = part<unsigned long long>(sc, kOffAcc) + (size_t)r * stride;
  const uint64_t* bnd = part<uint64_t>(sc, kOffBnd);
  const double nd0 = (double)part<int64_t>(sc, kOffNd0)[r];
  part<uint64_t>(sc, kOffOcc)[r] = bnd[r + 1] - bnd[r];
  part<uint64_t>(sc, kOffTot)[r] = a[0];
  const int64_t dre = (int64_t)a[1], dim = (int64_t)a[2];
  part<int64_t>(sc, kOffNdg)[2 * r] = dre;
  part<int64_t>(sc, kOffNdg)[2 * r + 1] = dim;
  part<double>(sc, kOffTr)[r] = (double)dre / nd0;
  part<double>(sc, kOffTh)[r] = atan2((double)dim, (double)dre);
  for (uint32_t k = 0; k < npl; ++k) {
    const int64_t pre = (int64_t)a[5 + 2 * k], pim = (int64_t)a[6 + 2 * k];
    part<int64_t>(sc, kOffPau)[((size_t)r * npl + k) * 2] = pre;
    part<int64_t>(sc, kOffPau)[((size_t)r * npl + k) * 2 + 1] = pim;
    part<double>(sc, kOffPv)[((size_t)r * npl + k) * 2] = (double)pre / nd0;
    part<double>(sc, kOffPv)[((size_t)r * npl + k) * 2 + 1] = (double)pim / nd0;
  }
  part<uint64_t>(sc, kOffEps2)[2 * r] = a[3];
  part<uint64_t>(sc, kOffEps2)[2 * r + 1] = a[4];
  part<double>(sc, kOffEps)[r] =
      sqrt((double)a[4] * 18446744073709551616.0 + (double)a[3]) / nd0;
  const double* pre = part<double>(sc, kOffPre);
  const double* pim = part<double>(sc, kOffPim);
  const int64_t* look = part<int64_t>(sc, kOffLout);
  double fre = 0.0, fim = 0.0;
  size_t idx = 0;
  for (uint32_t u = 0; u < npsi; ++u)
    for (uint32_t v = 0; v < npsi; ++v, ++idx) {
      const double ur = pre[u], ui = pim[u], vr = pre[v], vi = pim[v];
      const double pr = ur * vr + ui * vi, pi = ur * vi - ui * vr;
      const double A = (double)look[((size_t)r * nlook + idx) * 2];
      const double B = (double)look[((size_t)r * nlook + idx) * 2 + 1];
      fre += pr * A - pi * B;
      fim += pr * B + pi * A;
    }
  part<double>(sc, kOffFid)[2 * r] = fre / nd0;
  part<double>(sc, kOffFid)[2 * r + 1] = fim / nd0;
}

uint32_t replica_bits(uint32_t R) {
  uint32_t b = 0;
  while ((1ull << b) < R) ++b;
  return b;
}

}  // namespace

extern "C" int qmc_observe_noalloc(uint32_t n_qubits, uint32_t n_replicas, const uint64_t* d_keys,
                                   const int32_t* d_vals, uint64_t n, const int64_t* nd0_re,
                                   const qmc_obs_spec* spec, qmc_obs_out* out,
                                   void* hip_stream) {
  if (!spec || !out || n_qubits < 1 || n_qubits > 32 || n_replicas < 1 ||
      n_replicas > kNaReplicas || 2 * n_qubits + replica_bits(n_replicas) > 64)
    return QMC_ERR_ARG;
  if (n > 0 && (!d_keys || !d_vals)) return QMC_ERR_ARG;
  const uint32_t npl = spec->n_pauli, npsi = spec->n_psi, R = n_replicas;
  if (npl > kNaPauli || npsi > kNaPsi || (uint64_t)npsi * npsi * R > kNaLookTotal)
    return QMC_ERR_ARG;
  if ((npl && (!spec->px || !spec->pz)) ||
      (npsi && (!spec->psi_index || !spec->psi_re || !spec->psi_im)))
    return QMC_ERR_ARG;
  const uint64_t qmask = n_qubits >= 32 ? 0xFFFFFFFFull : ((1ull << n_qubits) - 1);
  for (uint32_t k = 0; k < npl; ++k)
    if ((spec->px[k] | spec->pz[k]) & ~qmask) return QMC_ERR_ARG;
  for (uint32_t u = 0; u < npsi; ++u)
    if (spec->psi_index[u] & ~qmask) return QMC_ERR_ARG;
  const bool fp = out->trace || out->theta || out->pauli_val || out->fidelity || out->eps;
  if (fp && !nd0_re) return QMC_ERR_ARG;

  hipStream_t st = (hipStream_t)hip_stream;
  uint8_t* sc = nullptr;
  if (scratch_of_current_device(&sc) != hipSuccess) return QMC_ERR_HIP;
  const uint32_t kbits = 2 * n_qubits;
  const uint32_t stride = 5 + 2 * npl;
#define NA_CHK(x)                                   \
  do {                                              \
    if ((hipError_t)(x) != hipSuccess) return QMC_ERR_HIP; \
  } while (0)
  // inputs: host arrays staged into the scratch
  if (npl) {
    NA_CHK(hipMemcpyAsync(sc + kOffPx, spec->px, 8 * (size_t)npl, hipMemcpyHostToDevice, st));
    NA_CHK(hipMemcpyAsync(sc + kOffPz, spec->pz, 8 * (size_t)npl, hipMemcpyHostToDevice, st));
  }
  if (npsi) {
    NA_CHK(hipMemcpyAsync(sc + kOffPidx, spec->psi_index, 8 * (size_t)npsi,
                          hipMemcpyHostToDevice, st));
    NA_CHK(hipMemcpyAsync(sc + kOffPre, spec->psi_re, 8 * (size_t)npsi, hipMemcpyHostToDevice,
                          st));
    NA_CHK(hipMemcpyAsync(sc + kOffPim, spec->psi_im, 8 * (size_t)npsi, hipMemcpyHostToDevice,
                          st));
  }
  if (nd0_re)
    NA_CHK(hipMemcpyAsync(sc + kOffNd0, nd0_re, 8 * (size_t)R, hipMemcpyHostToDevice, st));
  const uint32_t nacc = R * stride;
  hipLaunchKernelGGL(k_na_prepare, dim3(std::min<uint32_t>((nacc + kBlock - 1) / kBlock, 256u)),
                     dim3(kBlock), 0, st, sc, n, nacc, npl, npsi, n_qubits);
  NA_CHK(hipGetLastError());
  const int2* pv = reinterpret_cast<const int2*>(d_vals);
  void* cnt = sc + kOffCnt;
  NA_CHK(qmck_observe(st, d_keys, pv, cnt, 0, n_qubits, kbits, R, npl,
                      part<uint64_t>(sc, kOffPxz), spec->want_eps ? 1u : 0u,
                      part<unsigned long long>(sc, kOffAcc), stride, n));
  if (npsi)
    NA_CHK(qmck_lookup(st, d_keys, pv, cnt, 0, kbits, part<uint64_t>(sc, kOffLook), npsi * npsi,
                       R, part<int64_t>(sc, kOffLout)));
  NA_CHK(qmck_replica_bounds(st, d_keys, cnt, kbits, R, part<uint64_t>(sc, kOffBnd)));
  hipLaunchKernelGGL(k_na_finish, dim3((R + kBlock - 1) / kBlock), dim3(kBlock), 0, st, sc, R,
                     npl, npsi);
  NA_CHK(hipGetLastError());
  // outputs straight into the caller's arrays
  auto back = [&](void* dst, size_t off, size_t bytes) -> hipError_t {
    if (!dst || bytes == 0) return hipSuccess;
    return hipMemcpyAsync(dst, sc + off, bytes, hipMemcpyDeviceToHost, st);
  };
  NA_CHK(back(out->n_occ, kOffOcc, 8 * (size_t)R));
  NA_CHK(back(out->n_tot, kOffTot, 8 * (size_t)R));
  NA_CHK(back(out->ndiag, kOffNdg, 16 * (size_t)R));
  NA_CHK(back(out->pauli, kOffPau, 16 * (size_t)R * npl));
  NA_CHK(back(out->eps2, kOffEps2, 16 * (size_t)R));
  NA_CHK(back(out->trace, kOffTr, 8 * (size_t)R));
  NA_CHK(back(out->theta, kOffTh, 8 * (size_t)R));
  NA_CHK(back(out->pauli_val, kOffPv, 16 * (size_t)R * npl));
  NA_CHK(back(out->fidelity, kOffFid, 16 * (size_t)R));
  NA_CHK(back(out->eps, kOffEps, 8 * (size_t)R));
  NA_CHK(hipStreamSynchronize(st));
#undef NA_CHK
  return QMC_OK;
}
