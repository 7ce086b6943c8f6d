// Launch interface of the frame kernels (host side).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "circuit.h"

namespace stimgpu {

struct FrameParams {
  const DevOp *ops;             // the program; with event ops when ring != NULL
  uint32_t num_ops;
  uint32_t num_qubits;
  const uint32_t *targets;
  const uint64_t *thresholds;   // [rows][64]
  const uint64_t *ref;          // reference bits; NULL: write raw flips
  uint64_t seed;
  uint64_t word0;               // absolute word index of local word 0
  uint64_t num_words;           // W
  uint64_t tail_mask;           // valid bits of local word W - 1
  uint64_t *out;                // [M][out_stride]
  uint64_t out_stride;
  uint64_t *scratch;            // global frame slices when not in LDS
  // Precomputed noise (k_noise_gen), or noise_meta == NULL to draw it inline.
  // noise_meta[tile][execution] (walks with noz set, and batched walks) or
  // noise_meta[execution][noise_tiles] (otherwise) = {record count
  // (kNoRecords: draw inline),
  // index of the first record in noise_rec}.
  const uint2 *noise_meta;
  const uint4 *noise_rec;       // 16-byte records
  uint32_t noise_tiles;
  uint32_t noise_instances;
  // Detection events formed in the walk (ring != NULL): measurements write
  // their flips into the workgroup's ring of ring_rows rows of T words (slot
  // s at ring + s ring_rows T) instead of `out`; detector ops write rows of
  // det_out, observable ops XOR into rows of obs_out (NULL: skipped; its
  // num_obs rows are cleared first), both with row stride out_stride.
  uint64_t *ring;
  uint64_t *det_out;
  uint64_t *obs_out;
  uint32_t ring_rows;
  uint32_t num_obs;
  // The program is the one without Z randomisations (its walk honours the
  // flags that program carries).
  bool noz;
};

// Record count meaning "draw this noise op inline".
constexpr uint32_t kNoRecords = 0xFFFFFFFFu;
// LDS queue entries of one k_noise_gen workgroup (shared by its tiles), and
// the most tiles one workgroup takes.
constexpr uint32_t kGenQueue = 4096;
constexpr uint32_t kGenTiles = 16;

struct NoiseGenParams {
  const DevOp *ops;
  const uint32_t *targets;
  const uint64_t *thresholds;
  const uint32_t *inst_pc;      // [instances] pc of each noise execution
  const uint64_t *inst_instr;   // [instances] its flat instruction index
  const uint64_t *base;         // [instances]
  const uint32_t *cap;          // [instances] 0: leave to the walker
  uint64_t seed, word0, num_words;
  uint32_t tiles;
  // Entry (tile t, execution e) at meta[t * tile_stride + e * inst_stride]:
  // tile-major (inst_stride 1, tile_stride >= instances) for walks of the
  // program without Z randomisations, else execution-major (tile_stride 1,
  // inst_stride >= tiles); see FrameParams::noise_meta.
  uint32_t tile_stride, inst_stride;
  uint32_t tiles_per_group;     // tiles per workgroup (at most kGenTiles)
  uint32_t queue_per_tile;      // LDS queue entries per tile (tiles_per_group * this <= kGenQueue)
  uint2 *meta;                  // {count, first record}
  uint4 *rec;
};

// Fills the records of every (noise execution, tile); grid (tile groups,
// instances), `threads` (a multiple of 64, at most 512) per workgroup.
hipError_t launch_noise_gen(const NoiseGenParams &g, int tile_words, uint32_t instances, uint32_t threads,
                            hipStream_t stream);

struct FrameConfig {
  int tile_words;               // T: 1, 2, 4, 8, 16 or 32
  bool in_lds;
  uint32_t threads;
  uint32_t slots = 0;           // workgroups (global frame or ring slots); 0 = one per tile
  bool wave = false;            // batched launches: one wave per tile (k_batch_wave)
};

// LDS available to one workgroup on gfx950.
constexpr size_t kMaxLdsBytes = 160 * 1024;

// Dynamic LDS of one frame workgroup: a 64-entry queue per wave, one
// 64-entry threshold row, plus the frame slice (16 (n + 1) T bytes: the
// qubits and a dummy row) when it is held
// in LDS.
size_t frame_lds_bytes(uint64_t n, int T, bool in_lds, uint32_t threads);

hipError_t launch_frame(const FrameParams &p, const FrameConfig &cfg, hipStream_t stream);

// One unit of work of a batched launch: tile `tile` of request `req`.
struct BatchItem {
  uint32_t req;
  uint32_t tile;
};

// Static LDS of the batch kernel (the popped item index), kept out of the
// dynamic budget.
constexpr size_t kBatchStaticLds = 64;

// Resets *counter and launches the persistent batch kernel (LDS-resident
// frames, tile width cfg.tile_words in {1, 2, 4, 8}) over `blocks` workgroups.
hipError_t launch_batch(const FrameParams *reqs, const BatchItem *items, uint32_t num_items, uint32_t *counter,
                        const FrameConfig &cfg, uint64_t max_qubits, uint32_t blocks, hipStream_t stream);
// Workgroups of the batch kernel that fit on one CU at once.
int batch_blocks_per_cu(const FrameConfig &cfg, uint64_t max_qubits);
// One-wave-per-tile batches: LDS of one wave's tile (queue, threshold row,
// frame slice of n + 1 rows), and the waves of one workgroup (at most 16; 0
// when one wave's tile does not fit).
size_t wave_lds_bytes(uint64_t n, int T);
uint32_t batch_waves_per_block(uint64_t n, int T);
// Detection events / observable flips: row r of `out` = XOR of the flip rows
// idx[off[r] .. off[r+1]).  Rows are visited in `order` (NULL: 0, 1, ...).
hipError_t launch_parity(const uint64_t *flips, uint64_t W, const uint32_t *off, const uint32_t *idx,
                         const uint32_t *order, uint32_t rows, uint64_t *out, hipStream_t stream);
// Detection events by detector blocks (Program::det_blocks, nblocks of them).
hipError_t launch_parity_blocks(const uint64_t *flips, uint64_t W, const uint32_t *blocks, uint64_t nblocks,
                                const uint32_t *off, const uint32_t *idx, uint64_t *out, hipStream_t stream);

}  // namespace stimgpu
