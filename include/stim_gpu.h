/*
 * stim_gpu.h -- C ABI of the MI355X batched Pauli-frame sampler.
 *
 * The library implements the bulk-sampling path of Gidney, "Stim: a fast
 * stabilizer circuit simulator" (arXiv:2103.02202):
 *   - circuits in the line format of Sec. 5.10 (one operation per line,
 *     '#' comments, broadcasting over targets, REPEAT N { ... });
 *   - one noiseless reference sample from an inverse stabilizer tableau
 *     (Sec. 4), computed on the host;
 *   - Pauli-frame simulation of many shots at once (Sec. 3) on the GPU, with
 *     the frame stored as one bit per shot, shots along the fast axis
 *     (Sec. 5.1), X bits and Z bits in separate planes;
 *   - measurement results = reference XOR frame x bit (Sec. 3);
 *   - detection events = XOR of each detector's measurement flips (Sec. 5.6).
 *
 * Output layout (all sampling calls): row-major [rows][W] uint64 words with
 * W = ceil(num_shots / 64).  Bit j of word w of a row is shot
 * shot_offset + 64 w + j, least significant bit first as in the b8 format of
 * Sec. 5.11; bits past num_shots are zero.
 *
 * Random bits: every random choice is a pure function of (seed, flat
 * instruction index, target slot, absolute 64-shot word), drawn from
 * Philox4x64-10.  Results therefore do not depend on how shots are split
 * across calls, tiles or launches: sampling shots [a, b) in one call gives the
 * same bits as the corresponding slice of a larger call.
 *
 * Ownership: the library owns circuit handles and the device copies cached in
 * them (one per device, uploaded on first use).  The caller owns every output
 * buffer and every stream.  All pointers named out_* are device pointers.
 *
 * Errors: every int-returning call returns STIM_OK (0) or a negative code and
 * sets a thread-local message readable with stim_last_error().  No C++
 * exception crosses this interface.
 *
 * Concurrency: compile and reference calls are synchronous host work.
 * Sampling calls enqueue work on `hip_stream` (a hipStream_t; NULL = the
 * legacy default stream) and return without waiting, except that the first
 * call on a device uploads the circuit (hipMemcpyAsync on that stream).  After
 * stim_reference_sample has run, a handle is read-only and may be used from
 * several streams at once.
 */
#ifndef STIM_GPU_H
#define STIM_GPU_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  STIM_OK = 0,
  STIM_E_PARSE = -1,        /* malformed circuit text; message has the line */
  STIM_E_INVALID_ARG = -2,  /* null / misaligned / out-of-range argument */
  STIM_E_OOM = -3,          /* host or device allocation failed */
  STIM_E_DEVICE = -4,       /* a HIP call failed */
  STIM_E_UNSUPPORTED = -5   /* unknown gate, non-Pauli channel, size limit */
};

typedef struct stim_circuit stim_circuit;   /* opaque, library-owned */

/* Parses and compiles circuit text (Sec. 5.10).  `text` need not be
 * NUL-terminated.  On success *out receives a new handle.  Supported:
 * I X Y Z H H_XY H_YZ S S_DAG SQRT_X SQRT_X_DAG SQRT_Y SQRT_Y_DAG CX CY CZ SWAP
 * R M MR X_ERROR Y_ERROR Z_ERROR DEPOLARIZE1 DEPOLARIZE2 DETECTOR
 * OBSERVABLE_INCLUDE TICK QUBIT_COORDS SHIFT_COORDS REPEAT (and the aliases
 * CNOT ZCX ZCY ZCZ H_XZ SQRT_Z SQRT_Z_DAG RZ MZ MRZ).  CX, CY and CZ also
 * accept a measurement-record control rec[-k] in place of the control qubit
 * (for CZ on either side): the Pauli X, Y or Z is applied to the other target
 * when that result is 1 (Sec. 3, tracking corrections); such a pair counts as
 * one gate target.  Unknown gates give STIM_E_UNSUPPORTED; syntax errors, a
 * record as the target of CX / CY, records on both sides, or a lookback before
 * the first measurement give STIM_E_PARSE. */
int stim_compile(const char *text, size_t len, stim_circuit **out);

/* Frees a handle and its device copies.  NULL is ignored.  The caller must
 * ensure no sampling call using the handle is still running. */
void stim_circuit_free(stim_circuit *c);

/* Sizes of the compiled circuit.  Any output pointer may be NULL.
 * num_gate_targets counts each one-qubit Clifford / R / M / MR target and each
 * two-qubit Clifford pair once (noise and annotations excluded). */
int stim_circuit_shape(const stim_circuit *c, uint64_t *num_qubits, uint64_t *num_measurements,
                       uint64_t *num_detectors, uint64_t *num_observables, uint64_t *num_gate_targets);

/* The canonical noiseless reference sample (Sec. 4, inverse tableau): every
 * random measurement result -- including the measurement implied by a reset --
 * is taken to be 0; deterministic results are what they are.  Computed on the
 * first call and cached in the handle.  ref_out: host buffer of
 * ceil(num_measurements / 64) uint64 words (bit m = measurement m), or NULL
 * to only compute and cache. */
int stim_reference_sample(stim_circuit *c, uint64_t *ref_out);

/* The same canonical reference sample computed on the GPU (Sec. 4 with the
 * inverse tableau in device memory: one wave per target for each Clifford
 * layer, deterministic results of a measurement layer read in parallel, the
 * random ones collapsed in order by one workgroup).  Always recomputes; the
 * result is cached in the handle if none is.  ref_out: host buffer as for
 * stim_reference_sample, or NULL.  Runs on `hip_stream` and waits for it.
 * The sampling calls use this path by themselves for circuits of 1,024 or
 * more qubits (environment STIM_GPU_REFERENCE = 0 / 1 forces host / GPU). */
int stim_reference_sample_gpu(stim_circuit *c, uint64_t *ref_out, void *hip_stream);

/* Samples measurement records of shots [shot_offset, shot_offset + num_shots)
 * (Sec. 3).  out_meas: device buffer [num_measurements][W] uint64.
 * shot_offset must be a multiple of 64; num_shots > 0.  Computes the reference
 * sample first if it is not cached yet. */
int stim_frame_sample(stim_circuit *c, uint64_t seed, uint64_t shot_offset, uint64_t num_shots,
                      uint64_t *out_meas, void *hip_stream);

/* Samples detection events (Sec. 5.6) and observable flips of the same shots.
 * out_det: device [num_detectors][W]; out_obs: device [num_observables][W] or
 * NULL.  Event = XOR of the detector's measurement flips (the reference bits
 * cancel because detectors are deterministic in the noiseless circuit).
 * The frame walk writes the flip record and a second kernel forms the
 * events.  When every detector and observable is deterministic (checked once
 * per circuit by the backward walk behind stim_error_sets), the walk skips the
 * Z randomisations after collapses: each would add to the events the detector
 * set of a Z error at that point, which is then empty, so the events are the
 * same bits (STIM_EVENT_ZRAND=1 keeps the draws); an M followed by an R of
 * the same qubits then resets them itself (M, R is MR without the draws).
 * With STIM_WALK_EVENTS=1 the walk forms the events itself from a
 * per-workgroup ring of its recent flips (longest detector, observable or
 * feedback lookback plus the largest measurement instruction, at most the
 * whole record, in rows of the tile's words) when those rings fit in 512 MiB.
 * Same bits either way. */
int stim_detector_sample(stim_circuit *c, uint64_t seed, uint64_t shot_offset, uint64_t num_shots,
                         uint64_t *out_det, uint64_t *out_obs, void *hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * arguments and results as stim_detector_sample, bit for bit, without any
 * allocation.  The flip table of the call (and, for circuits whose frame does
 * not fit in LDS, the frame slots) lives in a device array of 256 MiB that
 * the library holds on each device it runs on until the process ends; the
 * noise is drawn inside the frame kernel (no pre-pass records).  Calls that
 * need more scratch than that (about 8 (num_measurements + 1)
 * ceil(num_shots / 64) bytes) return STIM_E_UNSUPPORTED: split the shots.
 * The circuit must already be resident on the current device -- any earlier
 * allocating sampling call on this device uploads it -- else
 * STIM_E_INVALID_ARG.  Every call on one device shares that array: calls that
 * overlap on one device (several streams or threads) race and must be
 * serialised by the caller. */
int stim_detector_sample_noalloc(stim_circuit *c, uint64_t seed, uint64_t shot_offset, uint64_t num_shots,
                                 uint64_t *out_det, uint64_t *out_obs, void *hip_stream);

/* Sparse detection-event sampling (Sec. 5.6: draw the errors, XOR the sets
 * of detectors each one flips).  Same arguments, output layout and results as
 * stim_detector_sample: the errors are drawn from the frame sampler's own
 * random streams, so the events are bit-identical, while the work is one
 * generator call per 32 noise sites and 64 shots plus the errors themselves
 * instead of a pass over every gate.  The error sets are built on the host on
 * the first call (cached in the handle).  Returns STIM_E_UNSUPPORTED (message
 * in stim_last_error) when a detector or observable depends on a random
 * measurement outcome, for classically controlled Paulis, and for circuits
 * whose noise executions cannot be tabulated. */
int stim_sparse_detector_sample(stim_circuit *c, uint64_t seed, uint64_t shot_offset, uint64_t num_shots,
                                uint64_t *out_det, uint64_t *out_obs, void *hip_stream);

/* The error sets behind stim_sparse_detector_sample (host only, no GPU
 * needed).  Generators are numbered by noise execution in circuit order
 * (noise instructions with p > 0, unrolled), then slot, then X and Z of the
 * slot's first qubit and (two-qubit channels) of its second.  Generator g
 * flips lanes[offsets[g] .. offsets[g + 1]) in increasing order, lane d <
 * num_detectors being detector d and lane num_detectors + o observable o.
 * *num_sets and *num_entries (host) receive the sizes; offsets (num_sets + 1
 * uint32) and lanes (num_entries uint32) are host buffers filled when not
 * NULL.  Errors as stim_sparse_detector_sample. */
int stim_error_sets(stim_circuit *c, uint64_t *num_sets, uint64_t *num_entries, uint32_t *offsets,
                    uint32_t *lanes);

/* Device memory, in bytes, that one sampling call of num_shots shots takes
 * from the stream-ordered pool of the current device beyond the caller's
 * outputs, for admission control.  mode 0: stim_frame_sample (noise records
 * of the pre-pass and their tables; the per-workgroup frame slots of circuits
 * too large for LDS); mode 1: stim_detector_sample (the same plus the flip
 * rings when the walk forms the events, else the flip table, one
 * ceil(num_shots / 64)-word row per measurement); mode 2:
 * stim_sparse_detector_sample (0: it allocates nothing per call).  Host only;
 * *bytes (host) receives the size.  STIM_E_INVALID_ARG for a null argument or
 * another mode. */
int stim_sample_scratch_bytes(stim_circuit *c, uint64_t num_shots, int mode, uint64_t *bytes);

/* One request of a batched launch. mode 0: out0 = measurement record
 * (as stim_frame_sample); mode 1: out0 = detection events, out1 = observable
 * flips or NULL (as stim_detector_sample). */
typedef struct {
  stim_circuit *c;
  uint64_t seed, shot_offset, num_shots;
  int mode;
  uint64_t *out0, *out1;
} stim_request;

/* Samples many requests (different circuits, shot counts and modes) in one
 * persistent launch on `hip_stream`; bit-identical to calling the single-
 * request functions one by one.  A request set seen for the first time runs
 * as one launch at an untuned (or previously tuned) shot-tile width; the
 * second submission of the same set (same handles, seeds, shots and output
 * pointers) times each candidate tile width x workgroup size on it, keeps
 * the fastest for its shape class (qubit count, total words and request
 * count, each rounded up to a power of two) and captures the launch in a HIP
 * graph that later submissions replay.  Environment: STIM_TUNE=0 skips the
 * timing trials; STIM_TUNE_CACHE=<file> keeps tuned shape classes across
 * processes (read on the first batched call, appended as classes are tuned).
 * A tuned width is reused only where the request set's largest frame fits
 * in LDS at that width. */
int stim_batch_sample(const stim_request *reqs, size_t n, void *hip_stream);

/* Shot-major output formats (Sec. 5.11, "Output Format"). */
enum {
  STIM_FORMAT_01 = 0,    /* '0'/'1' per result, '\n' after each shot: rows + 1 bytes per shot */
  STIM_FORMAT_B8 = 1,    /* 8 results per byte, LSB first, zero-padded: ceil(rows / 8) bytes per shot */
  STIM_FORMAT_HITS = 2,  /* indices of the set results in decimal, ',' between, '\n' after each shot */
  STIM_FORMAT_R8 = 3     /* per set result the zero run before it as bytes (255 = 255 zeros, continue),
                            then the zero run to the end of the shot the same way */
};

/* Writes shots [0, num_shots) of a measurement-major table in a shot-major
 * format (the two sparse formats, hits and r8, are this library's reading of
 * the formats the paper names without defining).  table: device
 * [rows][ceil(num_shots / 64)] uint64 as the samplers write it (a record,
 * events or observables); out: device buffer of out_cap bytes, or NULL with
 * out_cap 0 to only ask for the size.  *out_len (host) receives the number of
 * bytes of the whole output.  Dense formats (01, b8) have a fixed size and the
 * call is asynchronous on `hip_stream`; sparse formats (hits, r8) are sized by
 * a counting pass, so the call waits for the stream.  Returns
 * STIM_E_INVALID_ARG (writing nothing) if out_cap < *out_len, and for an 01
 * or b8 output that is not 4-byte aligned. */
int stim_format_shots(const uint64_t *table, uint64_t rows, uint64_t num_shots, int format, uint8_t *out,
                      uint64_t out_cap, uint64_t *out_len, void *hip_stream);

/* Per-kernel timing of sampling passes (stim_frame_sample and
 * stim_detector_sample; not batched launches).  stim_kernel_timing(1) discards
 * what was collected and starts recording HIP events on each pass's stream
 * around its noise pre-pass kernel and its frame kernel (at most 4096 passes
 * are kept); stim_kernel_timing(0) discards and stops.  stim_kernel_times
 * waits for the recorded passes, writes the summed durations in milliseconds
 * and the number of passes (any pointer may be NULL) and discards them;
 * recording stays on.  Passes without a pre-pass add 0 to noise_gen_ms. */
int stim_kernel_timing(int enable);
int stim_kernel_times(double *noise_gen_ms, double *frame_ms, uint64_t *passes);

/* Thread-local message of the last failing call ("" if none). */
const char *stim_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* STIM_GPU_H */
