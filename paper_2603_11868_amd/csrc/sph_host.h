// Host execution of the step (SPH_POLICY_HOST): the per-particle and per-pair
// bodies of sph_bodies.h run over host arrays on the CPU's threads, in the
// order the GPU path uses (cells in key order, sources of a target in the
// order of the direct search), FP64 only.  The paper's execution policies run
// one kernel source sequentially, in parallel on the host or on a device
// (Sec. 4); this is the host policy of the same bodies.  It is selected only by
// sph_params.policy and never stands in for the device path.
#pragma once

#include <stdint.h>

#include <vector>

#include "sph.h"
#include "sph_device.h"

namespace sphx {

class HostExec {
public:
    HostExec(const SimConst &sc, const std::vector<InstDev> &inst, int reorder_every, int nthreads);
    // Keep the caller's buffers (host memory) and build the wall table.
    void bind(const sph_buffers &b);
    void prime();
    void step();
    uint32_t flags() const { return flags_; }
    void clear_flags() { flags_ = 0; }
    int64_t steps_done() const { return steps_; }

private:
    template <int DIM> void keys(bool kick_on);
    void sort(bool reorder);
    template <int DIM> void pack();
    template <int DIM> void density(bool use_dt);
    template <int DIM> void force(bool fused);
    void reduce(bool prime);
    template <class F> void for_slots(F &&f) const;

    SimConst sc_;
    std::vector<InstDev> inst_;
    std::vector<int64_t> fo_;          // fluid offsets of the instances (B + 1)
    int K_;
    int nthreads_;
    sph_buffers buf_{};
    int64_t N_ = 0, Nw_ = 0, C_ = 0;
    std::vector<int> skey_, cnt_, wkey_, clamped_;
    std::vector<double> xs_, vs_, rhos_, Ps_, xws_;   // sorted copies (sources)
    std::vector<double> vals_;                        // per-particle diagnostics [N * kNPart]
    uint32_t flags_ = 0;
    int64_t steps_ = 0;
};

}  // namespace sphx
