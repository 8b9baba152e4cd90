// The row-OR stream of small networks on one wavefront per word column
// (Sec. 3.1 Algorithm 1 in reverse time, Sec. 3.4), and of many such
// networks in one launch (the hashed proxies, Sec. 4.3).
#pragma once

#include "tn_internal.h"

namespace tn {

// Small networks: the row-OR stream of one-word slices with the column in
// LDS, one wavefront per word column and no barrier (k_rowor_wave), for n
// real plus scratch rows in kRoworWaveLds bytes.  It loads and stores C
// once and keeps persist (as launch_rowor_global's with one-word slices)
// when given; traffic counts those loads and stores.  With saturation a
// column stops once every real row of it is all ones.
constexpr size_t kRoworWaveLds = 64 * 1024;
bool rowor_wave_fits(uint32_t n, uint32_t scratch_rows);
// ... and whether it beats the workgroup kernel: its lanes take a level's
// ops 64 at a time, one LDS round trip per 64, so it wins while levels are
// short (timed on ER networks with Poisson events: 199 and 460 ops per
// level, 2.2x and 1.25x faster; 736 ops per level, even)
constexpr int64_t kRoworWaveOpsPerLevel = 640;
bool rowor_wave_pays(uint32_t n, uint32_t scratch_rows, int64_t ops, int64_t levels);
// One network of a multi-network wavefront launch (the hashed proxies): its
// op schedule, its matrix (n rows of ld words) and its per-column state
// (nullable; the layout of launch_rowor_global's with one-word slices).
struct WaveNet {
    DevOps s;
    uint64_t *C;
    int64_t ld;
    uint32_t *persist;
};
// Levels average more than this many ops: each lane takes two ops of a
// level per LDS round trip (a group of 128) instead of one.
constexpr int64_t kRoworWaveWideOps = 80;
bool rowor_wave_wide(int64_t ops, int64_t levels);
// count networks of n nodes each, one wavefront per word column of each;
// nets: DEVICE array; scratch rows up to max_scratch_rows in every network;
// wide as rowor_wave_wide says for their schedules together.
hipError_t launch_rowor_wave_multi(const WaveNet *nets, uint32_t count, uint32_t n,
                                   uint32_t max_scratch_rows, bool wide,
                                   unsigned long long *traffic, bool saturation,
                                   unsigned int *done_count, hipStream_t st);
hipError_t launch_rowor_wave(const DevOps &s, uint32_t n, uint64_t *C, int64_t ld,
                             uint32_t scratch_rows, unsigned long long *traffic, bool saturation,
                             uint32_t *persist, unsigned int *done_count, hipStream_t st);

// Flat schedules of many networks (k_rowor_wave_flat): ops in level order
// as {a, b, d1, d2} LDS byte offsets of the rows in a column (n real rows,
// then the scratch rows; kFlatNone for no second target), with kFlatEnd set
// in a on the last op of each level.  The DevOps of a WaveNet then holds
// only ops and nops.
constexpr uint32_t kFlatEnd = 0x80000000u;
constexpr uint32_t kFlatOffMask = 0x7fffffffu;
constexpr uint32_t kFlatNone = 0xffffffffu;
// Writes the flat form of schedule s of a network of n nodes to out
// (4 uint32 per op, flat_ops_bytes(s) bytes).
size_t flat_ops_bytes(const HostSchedule &s);
void flat_ops_pack(const HostSchedule &s, uint32_t n, uint32_t *out);
// traffic (nullable) counts the row words loaded and stored, as for
// launch_rowor_wave.
hipError_t launch_rowor_wave_flat(const WaveNet *nets, uint32_t count, uint32_t n,
                                  uint32_t max_scratch_rows, bool saturation,
                                  unsigned int *done_count, unsigned long long *traffic,
                                  hipStream_t st);
// One network (a resident plan): flat_ops a DEVICE array of nops flat ops;
// C as for launch_rowor_wave, no per-column state; traffic nullable.
hipError_t launch_rowor_wave_flat1(const uint32_t *flat_ops, uint32_t nops, uint32_t n,
                                   uint64_t *C, int64_t ld, uint32_t scratch_rows,
                                   unsigned long long *traffic, bool saturation, hipStream_t st);

}  // namespace tn
