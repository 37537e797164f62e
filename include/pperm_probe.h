/*
 * pperm_probe.h -- measured ceilings of the resources the growth kernel uses
 * (libpperm.so).
 *
 * The method's hot path is no dense contraction and no stream: its steps
 * issue 32-bit vector ALU work, read and write the per-walk tables in LDS, and
 * read the pooled sums through L2.  The rooflines it is reported against are
 * measured on the device itself by the microbenchmarks of this call, not
 * taken from a data sheet.  Beside the three resources, two probes measure
 * how many instructions a SIMD issues when every wave's stream is scalar, or
 * alternates vector and scalar instructions as a walk-step's stream does
 * (about half of each), independent of each other or each feeding the next.
 */
#ifndef PPERM_PROBE_H
#define PPERM_PROBE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pperm_probe_result {
    double valu_lane_ops_per_s;   /* 32-bit VALU lane-operations per second, whole device      */
    double lds_bytes_per_s;       /* LDS bytes read per second, whole device (b128 reads)      */
    double l2_bytes_per_s;        /* bytes read per second from an L2-resident buffer          */
    double valu_ms, lds_ms, l2_ms; /* duration of each timed launch                            */
    uint32_t compute_units;       /* CUs the launches were sized for                           */
    uint32_t l2_buffer_bytes;     /* size of the L2-resident buffer that was read              */
    double salu_instr_per_s;      /* wave instructions per second, scalar ALU only, whole device */
    double mixed_instr_per_s;     /* wave instructions per second, vector and scalar ALU
                                     alternating in each wave, whole device                    */
    double salu_ms, mixed_ms;     /* duration of each timed launch                            */
    uint32_t clock_khz;           /* the device's peak engine clock (HIP attribute), kHz       */
    uint32_t simds;               /* SIMDs the issue rates are spread over (4 per CU)          */
    double dependent_instr_per_s; /* wave instructions per second, vector compares feeding
                                     scalar mask and count instructions feeding vector adds,
                                     eight waves per SIMD, whole device                        */
    double dependent4_instr_per_s; /* the same with four waves per SIMD                        */
    double dependent_ms, dependent4_ms; /* duration of each timed launch                       */
} pperm_probe_result;

/* Run the probes on the current device, in order (VALU, LDS, L2, scalar
 * issue, mixed issue, dependent issue at eight and at four waves per SIMD), on
 * hip_stream (NULL: the default stream), each once untimed and once timed with
 * HIP events, and synchronise.  The issue probes run eight waves per SIMD (the
 * last one four), each wave with two or more chains, and count the
 * instructions of their unrolled bodies only (loop control excluded, so the
 * rates are slight underestimates).  d_buffer: caller-owned scratch device
 * memory of at least 1 MiB (PPERM_PROBE_BUFFER_BYTES), 256-byte aligned, whose
 * contents do not matter: the L2 probe reads its first MiB, and each probe
 * keeps its work live with a store into the first 256 bytes that happens only
 * when a checksum of what it read equals one fixed value.  *out receives the
 * ceilings.  Errors: PPERM_EINVAL (-1) for a null, short or misaligned buffer,
 * PPERM_EDEVICE (-3) for a failed HIP call. */
#define PPERM_PROBE_BUFFER_BYTES (1u << 20)
int pperm_probe(void* d_buffer, size_t bytes, void* hip_stream, pperm_probe_result* out);

#ifdef __cplusplus
}
#endif

#endif /* PPERM_PROBE_H */
