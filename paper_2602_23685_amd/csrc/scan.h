// Internal interface of the insertion scan, used by the ALNS driver.
#pragma once

#include "common.h"

namespace vrprpd {

struct ScanArgs {
    const InstDev* inst_tab;
    const void* dist;
    const int32_t* proc;
    const int32_t* base_inst;
    const int64_t* base_op_off;
    const uint16_t* base_ops;
    const int64_t* base_rt_off;
    const uint16_t* base_rt_end;
    const int64_t* seg_off;
    const int32_t* seg_base;
    const vrprpd_tuple* tuples;
    int32_t* mk_out;
    uint32_t* st_out;
    int64_t* seg_top3;
    const int32_t* seg_cnt;   // internal: segment s covers [seg_off[s], seg_off[s] + seg_cnt[s])
    int32_t num_bases, num_inst, n_max, num_seg;
    int32_t blocks_per_seg;   // blocks sharing one segment's tuples (>= 1)
    int32_t top3_ready = 0;   // internal: seg_top3 already holds INT64_MAX (no fill launch)
    // internal: with seg_active > 0 the launch covers only the first
    // seg_active segments of each group of seg_stride (num_seg = groups *
    // seg_active): block x scans segment (x / seg_active) * seg_stride + x % seg_active
    int32_t seg_active = 0, seg_stride = 0;
};

// Launches the insertion-scan kernel for the arguments above.
int insert_scan_launch(const ScanArgs& a, int m_max, int dist16, hipStream_t st);

}  // namespace vrprpd
