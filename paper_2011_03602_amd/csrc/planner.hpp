// Transfer planner: which arrays move between host and device, and when, for
// a given offload gene. A pure function of (gene, placement mode, validity
// state); the executor and ofl_plan() both use it, so what is tested on the
// CPU is what runs.
//
// Rules (paper Sec. 4.2.2): a variable that the CPU side set and a GPU nest
// references moves host->device; a variable a GPU nest set and the CPU side
// references (or sets) moves device->host. Placement (Sec. 3.2.1): in the
// hoisted mode a variable moves only when the side about to use it has no
// valid copy, so invariant inputs move once, outside the loop; in the
// per-iteration mode every GPU nest copies in all it reads and copies out all
// it writes, each time.
//
// Nest read/write sets of the Jacobi program:
//   S reads the 12 read-only arrays and p, writes wrk2 on the interior;
//   R reads p and wrk2 (writes only the scalar gosa);
//   C reads wrk2, writes p on the interior.
// A nest that writes only the interior of an array whose boundary layer is
// still live (p: its boundary is the Dirichlet data) must first hold the whole
// array on its side, so C also "reads" p. wrk2's boundary is never read by
// anyone, so S writes wrk2 without first fetching it.
#pragma once

#include <cstdint>
#include <vector>

#include "ofl.h"

namespace ofl {

struct Xfer {
    int iter, nest, when, array, dir;  // dir 0: host->device, 1: device->host
};

struct Validity {
    uint8_t host[OFL_NARRAYS];
    uint8_t dev[OFL_NARRAYS];
};

inline Validity fresh_validity() {
    Validity v;
    for (int a = 0; a < OFL_NARRAYS; ++a) {
        v.host[a] = 1;
        v.dev[a] = 0;
    }
    return v;
}

inline int nest_reads(int nest, int *out) {
    int n = 0;
    if (nest == 0) {
        for (int a = 0; a < 12; ++a)
            out[n++] = a;
        out[n++] = OFL_ARR_P;
    } else if (nest == 1) {
        out[n++] = OFL_ARR_P;
        out[n++] = OFL_ARR_WRK2;
    } else {
        out[n++] = OFL_ARR_WRK2;
        out[n++] = OFL_ARR_P;  // interior-only write of an array with a live boundary
    }
    return n;
}

inline int nest_writes(int nest) {
    if (nest == 0)
        return OFL_ARR_WRK2;
    if (nest == 2)
        return OFL_ARR_P;
    return -1;
}

// Transfers needed before nest `nest` runs on the GPU (gpu) or the CPU.
inline void plan_before(int iter, int nest, bool gpu, int mode, Validity &v, std::vector<Xfer> &out) {
    int reads[16];
    const int n = nest_reads(nest, reads);
    for (int t = 0; t < n; ++t) {
        const int a = reads[t];
        if (gpu) {
            // Never overwrite a newer device copy with a stale host copy.
            const bool need = v.host[a] && (mode == OFL_XFER_PER_ITER || !v.dev[a]);
            if (need) {
                out.push_back({iter, nest, 0, a, 0});
                v.dev[a] = 1;
            }
        } else if (!v.host[a]) {
            out.push_back({iter, nest, 0, a, 1});
            v.host[a] = 1;
        }
    }
}

// State change (and per-iteration copy-out) after nest `nest` ran.
inline void plan_after(int iter, int nest, bool gpu, int mode, Validity &v, std::vector<Xfer> &out) {
    const int a = nest_writes(nest);
    if (a < 0)
        return;
    if (gpu) {
        v.dev[a] = 1;
        v.host[a] = 0;
        if (mode == OFL_XFER_PER_ITER) {
            out.push_back({iter, nest, 1, a, 1});
            v.host[a] = 1;
        }
    } else {
        v.host[a] = 1;
        v.dev[a] = 0;
    }
}

// Arrays the GPU nests of `mask` read that are inputs of the loop (the twelve
// read-only arrays and the initial iterate): what a data region copies in up
// front.
inline void plan_enter(unsigned mask, Validity &v, std::vector<Xfer> &out) {
    if (mask == 0)
        return;
    if (mask & OFL_NEST_SWEEP)
        for (int a = 0; a < 12; ++a)
            if (!v.dev[a] && v.host[a]) {
                out.push_back({-1, -1, 0, a, 0});
                v.dev[a] = 1;
            }
    if (!v.dev[OFL_ARR_P] && v.host[OFL_ARR_P]) {
        out.push_back({-1, -1, 0, OFL_ARR_P, 0});
        v.dev[OFL_ARR_P] = 1;
    }
}

// p must be valid on the host once the caller reads it (after the loop).
inline void plan_sync_host(int iter, Validity &v, std::vector<Xfer> &out) {
    if (!v.host[OFL_ARR_P]) {
        out.push_back({iter, -1, 1, OFL_ARR_P, 1});
        v.host[OFL_ARR_P] = 1;
    }
}

}  // namespace ofl
