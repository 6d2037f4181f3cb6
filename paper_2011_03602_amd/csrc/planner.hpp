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
// A program is a sequence of loop nests inside the iteration loop, each given
// by the arrays it reads, the arrays it writes, and the arrays it writes only
// in part while the rest of the array stays live: such an array must be whole
// on the writer's side first, so it moves as if it were read. The planner
// works on any such table (ofl_plan_nests); the Jacobi program is one:
//   S reads the 12 read-only arrays and p, writes wrk2 on the interior;
//   R reads p and wrk2 (writes only the scalar gosa);
//   C reads wrk2, writes p on the interior.
// p's boundary layer is live (it is the Dirichlet data), so C writes p in
// part; wrk2's boundary is never read by anyone, so S's write of wrk2 is not
// partial and S writes it without first fetching it. The CPU program reads p
// after the loop.
#pragma once

#include <cstdint>
#include <vector>

#include "ofl.h"

namespace ofl {

constexpr int kMaxArrays = 32;
constexpr int kMaxNests = 8;

struct Xfer {
    int iter, nest, when, array, dir;  // dir 0: host->device, 1: device->host
};

struct Validity {
    uint8_t host[kMaxArrays];
    uint8_t dev[kMaxArrays];
};

inline Validity fresh_validity() {
    Validity v;
    for (int a = 0; a < kMaxArrays; ++a) {
        v.host[a] = 1;
        v.dev[a] = 0;
    }
    return v;
}

// Variables of one nest as bit sets over array ids.
struct NestVars {
    uint32_t reads, writes, partial;
};

struct Program {
    NestVars nests[kMaxNests];
    int nnests;
    int narrays;
    uint32_t live_after;  // arrays the CPU side references after the loop
};

inline const Program &jacobi_program() {
    static const Program prog = [] {
        Program p{};
        p.nnests = 3;
        p.narrays = OFL_NARRAYS;
        const uint32_t ro = (1u << 12) - 1u, P = 1u << OFL_ARR_P, W = 1u << OFL_ARR_WRK2;
        p.nests[0] = {ro | P, W, 0u};
        p.nests[1] = {P | W, 0u, 0u};
        p.nests[2] = {W, P, P};
        p.live_after = P;
        return p;
    }();
    return prog;
}

// Arrays a nest needs whole on its side before it runs, in the order they
// move: what it reads (ascending ids), then what it writes in part.
inline int nest_needs(const Program &prog, int nest, int *out) {
    const NestVars &n = prog.nests[nest];
    int c = 0;
    for (int a = 0; a < prog.narrays; ++a)
        if ((n.reads >> a) & 1u)
            out[c++] = a;
    for (int a = 0; a < prog.narrays; ++a)
        if (((n.partial >> a) & 1u) && !((n.reads >> a) & 1u))
            out[c++] = a;
    return c;
}

// Transfers needed before nest `nest` runs on the GPU (gpu) or the CPU.
inline void plan_before(const Program &prog, int iter, int nest, bool gpu, int mode, Validity &v,
                        std::vector<Xfer> &out) {
    int need[kMaxArrays];
    const int n = nest_needs(prog, nest, need);
    for (int t = 0; t < n; ++t) {
        const int a = need[t];
        if (gpu) {
            // Never overwrite a newer device copy with a stale host copy.
            const bool move = v.host[a] && (mode == OFL_XFER_PER_ITER || !v.dev[a]);
            if (move) {
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
inline void plan_after(const Program &prog, int iter, int nest, bool gpu, int mode, Validity &v,
                       std::vector<Xfer> &out) {
    const uint32_t w = prog.nests[nest].writes;
    for (int a = 0; a < prog.narrays; ++a) {
        if (!((w >> a) & 1u))
            continue;
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
}

// What a data region copies in up front: the arrays the GPU nests of `mask`
// need that are inputs of the loop body (needed before any nest wrote them).
inline void plan_enter(const Program &prog, unsigned mask, Validity &v, std::vector<Xfer> &out) {
    uint32_t in = 0, written = 0;
    for (int n = 0; n < prog.nnests; ++n) {
        const NestVars &x = prog.nests[n];
        if ((mask >> n) & 1u)
            in |= (x.reads | x.partial) & ~written;
        written |= x.writes;
    }
    for (int a = 0; a < prog.narrays; ++a)
        if (((in >> a) & 1u) && !v.dev[a] && v.host[a]) {
            out.push_back({-1, -1, 0, a, 0});
            v.dev[a] = 1;
        }
}

// The arrays the CPU side references after the loop must be valid there.
inline void plan_sync_host(const Program &prog, int iter, Validity &v, std::vector<Xfer> &out) {
    for (int a = 0; a < prog.narrays; ++a)
        if (((prog.live_after >> a) & 1u) && !v.host[a]) {
            out.push_back({iter, -1, 1, a, 1});
            v.host[a] = 1;
        }
}

// The Jacobi program's planner (what the executor runs).
inline void plan_before(int iter, int nest, bool gpu, int mode, Validity &v, std::vector<Xfer> &out) {
    plan_before(jacobi_program(), iter, nest, gpu, mode, v, out);
}
inline void plan_after(int iter, int nest, bool gpu, int mode, Validity &v, std::vector<Xfer> &out) {
    plan_after(jacobi_program(), iter, nest, gpu, mode, v, out);
}
inline void plan_enter(unsigned mask, Validity &v, std::vector<Xfer> &out) {
    plan_enter(jacobi_program(), mask, v, out);
}
inline void plan_sync_host(int iter, Validity &v, std::vector<Xfer> &out) {
    plan_sync_host(jacobi_program(), iter, v, out);
}

}  // namespace ofl
