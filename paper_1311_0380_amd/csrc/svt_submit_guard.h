// What a request leaves behind when its submission fails part way.
//
// A request enqueues copies and kernels on the caller's stream one call at a
// time.  When a later call fails, the commands already enqueued may still
// read or write the request's staging buffer, its scan scratch and its slot's
// host-mapped partial sums.  None of these may go to another request until
// the stream has finished them, so a failed submission that has enqueued
// anything waits for its stream before it gives its buffers back.  A
// submission that fails before its first enqueue gives them back at once; a
// submitted request keeps them until its completion is collected.
//
// Host-only and free of HIP types, so that the rule can be unit-tested on
// a machine without a GPU.
#pragma once
#include <utility>

namespace svt {

template <class Sync, class Release>
class SubmitGuard {
public:
    SubmitGuard(Sync sync, Release release) : sync_(std::move(sync)), release_(std::move(release)) {}
    SubmitGuard(const SubmitGuard &) = delete;
    SubmitGuard &operator=(const SubmitGuard &) = delete;
    ~SubmitGuard()
    {
        if (submitted_) return;
        if (enqueued_) sync_();
        release_();
    }
    // from here on commands of the request may be on the stream
    void enqueuing() { enqueued_ = true; }
    // the request is in flight: its completion releases the buffers
    void submitted() { submitted_ = true; }

private:
    Sync sync_;
    Release release_;
    bool enqueued_ = false, submitted_ = false;
};

template <class Sync, class Release>
SubmitGuard<Sync, Release> make_submit_guard(Sync sync, Release release)
{
    return SubmitGuard<Sync, Release>(std::move(sync), std::move(release));
}

}  // namespace svt
