// Process-wide arbitration of the persistent full -> band panel kernel.
//
// That kernel synchronises its whole grid (up to 64 workgroups) once per
// panel column, so all its workgroups must be resident at once.  Two such
// grids from concurrent solves on one device can each hold part of the
// device while waiting for the rest, until the kernel's wait bound.  The
// arbiter lets one handle per device own the persistent route at a time;
// every other solve on that device takes the per-column route, which needs
// no co-residency.  An owner keeps the route until its solve has finished
// on the device (the caller synchronises before releasing).
//
// Host-only C++ (no HIP), so the route selection is testable on any CPU.
#pragma once
#include <mutex>

namespace gevd {

class PanelArbiter {
   public:
    static constexpr int MAXDEV = 64;

    // True when `owner` now holds (or already held) the persistent route on
    // `device`; false when another owner holds it or the device index is
    // out of range.  Never blocks for long (a short critical section).
    bool try_acquire(int device, const void* owner) {
        if (device < 0 || device >= MAXDEV || !owner) return false;
        std::lock_guard<std::mutex> lk(mu_);
        if (owner_[device] == nullptr) {
            owner_[device] = owner;
            depth_[device] = 1;
            return true;
        }
        if (owner_[device] == owner) {
            ++depth_[device];
            return true;
        }
        return false;
    }

    // Releases one acquisition by `owner` (no effect if it does not own it).
    void release(int device, const void* owner) {
        if (device < 0 || device >= MAXDEV || !owner) return;
        std::lock_guard<std::mutex> lk(mu_);
        if (owner_[device] != owner) return;
        if (--depth_[device] <= 0) {
            owner_[device] = nullptr;
            depth_[device] = 0;
        }
    }

    const void* owner(int device) {
        if (device < 0 || device >= MAXDEV) return nullptr;
        std::lock_guard<std::mutex> lk(mu_);
        return owner_[device];
    }

   private:
    std::mutex mu_;
    const void* owner_[MAXDEV] = {};
    int depth_[MAXDEV] = {};
};

// The process's arbiter (one instance shared by all handles).
inline PanelArbiter& panel_arbiter() {
    static PanelArbiter a;
    return a;
}

}  // namespace gevd
