// Internal declarations shared by the host planner, the C ABI and the kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/tn.h"

namespace tn {

// Pair item encoding: {u, v | kDirBit}.  Undirected pair: both rows <- u | v.
// Directed pair (kDirBit set): row u <- u | v, row v unchanged.
constexpr uint32_t kDirBit = 0x80000000u;
constexpr uint32_t kNodeMask = 0x7fffffffu;

// A single network's schedule on the host.  Items are sorted by level;
// level l owns pairs [lvl_pair[l], lvl_pair[l+1]) and gathers
// [lvl_gat[l], lvl_gat[l+1]).  Gather g writes row gat_tgt[g] with the OR of
// rows gat_src[gat_ptr[g] .. gat_ptr[g+1]) read before any gather of its
// level writes.
struct HostSchedule {
    uint32_t n = 0;
    int64_t m = 0;
    uint32_t flags = 0;
    uint32_t L = 0;
    std::vector<uint32_t> lvl_pair;  // L + 1
    std::vector<uint32_t> lvl_gat;   // L + 1
    std::vector<uint32_t> pairs;     // 2 * P (u, v | dir)
    std::vector<uint32_t> gat_tgt;   // G
    std::vector<uint32_t> gat_ptr;   // G + 1
    std::vector<uint32_t> gat_src;   // S
    int64_t compound_items = 0;
    int64_t directed_pairs = 0;
    int64_t max_level_items = 0;
    int64_t max_level_gathers = 0;
    double host_seconds = 0.0;
};

// Device view of one schedule (all pointers into one allocation).
struct DevSchedule {
    uint32_t n;
    uint32_t L;
    uint32_t max_gat;      // widest level, in gathers
    uint32_t pad_;
    const uint32_t *lvl_pair;
    const uint32_t *lvl_gat;
    const uint2 *pairs;
    const uint32_t *gat_tgt;
    const uint32_t *gat_ptr;
    const uint32_t *gat_src;
};

// Validates events and builds the schedule.  Returns TN_OK or an error code
// with `err` set.
tn_status plan_events(uint32_t n, int64_t m, const uint32_t *src,
                      const uint32_t *dst, const int64_t *t, uint32_t flags,
                      HostSchedule &out, std::string &err);

// Size in bytes of the device image of a schedule and its packing.
size_t schedule_device_bytes(const HostSchedule &s);
void schedule_pack(const HostSchedule &s, std::vector<unsigned char> &image);
DevSchedule schedule_view(const HostSchedule &s, const void *dev_base);

// ---- kernel launchers (tn_kernels.hip) ---------------------------------
hipError_t launch_identity(uint64_t *C, uint32_t n, int64_t ld, hipStream_t st);
hipError_t launch_rowor_global(const DevSchedule &s, uint64_t *C, int64_t ld,
                               uint32_t slice_words, uint64_t *scratch,
                               hipStream_t st);
hipError_t launch_out_sizes(const uint64_t *C, uint32_t n, int64_t ld,
                            int32_t *out_sizes, hipStream_t st);
hipError_t launch_in_sizes(const uint64_t *C, uint32_t n, int64_t ld,
                           int32_t *in_sizes, hipStream_t st);
uint32_t default_slice_words(uint32_t n, int64_t ld);

}  // namespace tn
