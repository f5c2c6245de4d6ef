// Host-side launchers of the gfx950 kernels (defined in kernels.hip).
// Every launcher enqueues on `stream` and returns the hipError_t of the
// launch (hipSuccess on success).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "plan.h"

namespace svk {

using K2Args = svp::K2Args;

hipError_t init_zero_state(void *S, int n, int dtype, hipStream_t st);
// The state's storage order (sto in k2_device.h): every kernel addresses
// amplitude i at sto(i). plain_storage: the order is the identity for this
// size. to_storage_order: reorder a buffer given in plain order, in place.
bool plain_storage(int n, int dtype);
hipError_t to_storage_order(void *S, int n, int dtype, hipStream_t st);

// Batched passes: see k6_batch_kernel. grid must not exceed the resident
// capacity (k6_occupancy work-groups per CU times the CU count) so that the
// work-groups of one instance can wait for each other.
// lmax: the largest register tile of any instance (3..5; selects the
// build); mfma: some pass runs matrix-core windows. jobs: int2 (instance,
// rank) records, work-group w running wg_off[w] .. wg_off[w+1]-1.
int k6_max_threads(int dtype, int lmax);
int k6_occupancy(int dtype, int lmax, unsigned threads, size_t lds, bool mfma);
hipError_t k6_batch(int dtype, int lmax, unsigned grid, unsigned threads, size_t lds, const svp::BatchInst *insts,
                    const int32_t *wg_off, const void *jobs, const svp::BatchPass *passes, const svp::K2Op *ops,
                    unsigned *ctrs, int *err, unsigned limit, bool mfma, hipStream_t st);
hipError_t zero_u32(unsigned *p, uint32_t n, hipStream_t st);
hipError_t k1_gate(void *S, int n, int dtype, const svp::MGate &g, hipStream_t st);
hipError_t k3_swap(void *S, int n, int dtype, int p, int v, hipStream_t st);
// Extended gate: a k-qubit unitary U (device, 4^k amplitudes of the state's
// type, row-major, bit b of the row index = target b) on physical target bits
// tbits[0..k-1] where every physical bit cbits[0..nc-1] is 1 (k <= 6).
struct KqArg {
    int8_t fixed[24];   // targets and controls, ascending
    int32_t nfixed, k;
    uint64_t cmask;
    uint64_t toff[6];   // storage-order offset of each target bit
};
hipError_t kq_gate(void *S, int n, int dtype, const int *tbits, int k, const int *cbits, int nc, const void *U,
                   hipStream_t st);
// mfma: the op list holds matrix-core windows.
hipError_t k2_pass(void *S, int n, int dtype, int logr, const K2Args &a, const svp::K2Op *dev_ops, bool mfma,
                   hipStream_t st);

// Measurement. scan_inclusive: out[i] = in[0] + ... + in[i] in a fixed order
// (in == out allowed); scratch: scan_scratch_bytes(m). sample_outcomes: for
// each uniform u, the smallest m with cdf[m] > u * cdf[M - 1]. collapse: zero
// the amplitudes whose physical bits in mask differ from val, scale the rest.
size_t scan_scratch_bytes(uint64_t m);
hipError_t scan_inclusive(const double *in, double *out, uint64_t m, void *scratch, hipStream_t st);
hipError_t sample_outcomes(const double *cdf, uint64_t M, const double *u, uint64_t shots, uint64_t *out,
                           hipStream_t st);
hipError_t collapse(void *S, int n, int dtype, uint64_t mask, uint64_t val, double scale, hipStream_t st);

// Plain HBM stream (bandwidth reference): mode 0 copy, 1 in place.
hipError_t stream_probe(void *dst, const void *src, uint64_t bytes, int mode, hipStream_t st);

// Readouts (FP64). perm: HOST array of n ints, perm[q] = physical bit of
// logical bit q, or nullptr for the identity (passed to the kernel by value).
hipError_t probabilities(const void *S, int n, int dtype, const int *perm, double *out,
                         uint64_t offset, uint64_t count, hipStream_t st);
// Marginal over `nq` qubits given as physical bit positions (HOST array
// `qbits`, nq entries) and the complementary physical bits (`obits`, n-nq
// entries, ascending). out: 2^nq doubles on the device. scratch: at least
// marginal_scratch_bytes(n, nq) bytes of device memory.
size_t marginal_scratch_bytes(int n, int nq);
hipError_t marginal(const void *S, int n, int dtype, const int *qbits, int nq, const int *obits,
                    double *out, void *scratch, hipStream_t st);
// Argmax of a device FP64 array; lowest index wins ties. Result written to
// res[0] (index as double-punned uint64) and val[0]. scratch: argmax_scratch_bytes.
size_t argmax_scratch_bytes(uint64_t len);
hipError_t argmax(const double *p, uint64_t len, void *scratch, uint64_t *res_idx, double *res_val,
                  hipStream_t st);
// Fused marginal + argmax for marginals whose complement is small.
hipError_t marginal_argmax(const void *S, int n, int dtype, const int *qbits, int nq,
                           const int *obits, void *scratch, uint64_t *res_idx, double *res_val,
                           hipStream_t st);
// Device scratch that is never allocated: a file-scope array of
// static_scratch_bytes() per GPU, large enough for marginal_argmax's scratch
// (argmax_scratch_bytes) plus 256 bytes of results. static_scratch() returns
// its address on the current device (looked up once per device).
size_t static_scratch_bytes();
hipError_t static_scratch(void **out);
size_t norm_scratch_bytes(int n);
hipError_t norm2(const void *S, int n, int dtype, void *scratch, double *res, hipStream_t st);
// Logical-order gather: out[i] = S[phys(offset + i)] for i < count.
hipError_t gather_logical(const void *S, int n, int dtype, const int *perm, void *out,
                          uint64_t offset, uint64_t count, hipStream_t st);
hipError_t scatter_logical(void *S, int n, int dtype, const int *perm, const void *in,
                           uint64_t offset, uint64_t count, hipStream_t st);

}  // namespace svk
