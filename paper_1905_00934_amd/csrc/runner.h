// Slices of one precision grouped by shape: one launch per kernel per group, each
// covering every slice of the group through blockIdx.z.
#pragma once

#include <vector>

#include "kernels.h"

namespace dect {

template <typename T>
class Runner {
public:
    Runner() = default;
    Runner(const Runner&) = delete;
    Runner& operator=(const Runner&) = delete;
    ~Runner();

    // Group `jobs` by shape and launch structure (CG steps per iteration, rho mode;
    // slice order kept within a group) and copy their
    // argument blocks to device memory, which grows as needed and is reused.  The
    // copy is synchronous: no iteration enqueued earlier may still be running.
    hipError_t set(const std::vector<SliceJob<T>>& jobs);
    // One outer iteration of every slice, enqueued on s.
    hipError_t enqueue(hipStream_t s) const;
    // The dual rescale the iterations leave pending, applied to every slice's state
    // (launch_settle), enqueued on s.
    hipError_t settle(hipStream_t s) const;
    int groups() const { return (int)groups_.size(); }
    int slices() const { return n_; }

private:
    struct Group {
        std::vector<SliceJob<T>> jobs;
        JobArrays<T> dev{};
    };
    std::vector<Group> groups_;
    int n_ = 0;
    void* mem_ = nullptr;
    size_t cap_ = 0;
};

// Parameters a batched run accepts (fixed or adaptive rho, no schedule).
dect_status check_batch_params(const dect_params* prm);

}  // namespace dect
