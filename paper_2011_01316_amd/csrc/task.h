// A minimal C++20 coroutine task used by the Krylov controller.
//
// A Task<int> starts suspended.  Awaiting it from another task runs it and
// resumes the awaiter when it finishes (symmetric transfer, no recursion on
// the host stack).  A top-level task is started with resume(); when one of its
// awaits suspends, resume() returns and the executor keeps the suspended
// coroutine handle to resume later.  Allocation failure of a frame yields an
// empty task (valid() == false) instead of an exception.
#pragma once

#include <coroutine>
#include <exception>
#include <new>
#include <utility>

namespace expdg {

template <typename R>
class Task {
  public:
    struct promise_type {
        R value{};
        std::coroutine_handle<> cont;  // the awaiting coroutine (none at top level)

        Task get_return_object() noexcept {
            return Task(std::coroutine_handle<promise_type>::from_promise(*this));
        }
        static Task get_return_object_on_allocation_failure() noexcept { return Task(); }
        static void *operator new(std::size_t n) noexcept { return ::operator new(n, std::nothrow); }
        static void operator delete(void *p) noexcept { ::operator delete(p); }
        std::suspend_always initial_suspend() noexcept { return {}; }
        struct Final {
            bool await_ready() noexcept { return false; }
            std::coroutine_handle<> await_suspend(
                std::coroutine_handle<promise_type> h) noexcept {
                std::coroutine_handle<> c = h.promise().cont;
                return c ? c : std::noop_coroutine();
            }
            void await_resume() noexcept {}
        };
        Final final_suspend() noexcept { return {}; }
        void return_value(R v) noexcept { value = v; }
        void unhandled_exception() noexcept { std::terminate(); }
    };

    Task() = default;
    Task(const Task &) = delete;
    Task &operator=(const Task &) = delete;
    Task(Task &&o) noexcept : h_(std::exchange(o.h_, {})) {}
    Task &operator=(Task &&o) noexcept {
        if (this != &o) {
            if (h_) h_.destroy();
            h_ = std::exchange(o.h_, {});
        }
        return *this;
    }
    ~Task() {
        if (h_) h_.destroy();
    }

    bool valid() const { return (bool)h_; }
    bool done() const { return h_ && h_.done(); }
    void start() { h_.resume(); }
    R result() const { return h_.promise().value; }

    // awaiting a task runs it to completion (possibly across suspensions)
    bool await_ready() const noexcept { return false; }
    std::coroutine_handle<> await_suspend(std::coroutine_handle<> c) noexcept {
        h_.promise().cont = c;
        return h_;
    }
    R await_resume() const noexcept { return h_.promise().value; }

  private:
    explicit Task(std::coroutine_handle<promise_type> h) : h_(h) {}
    std::coroutine_handle<promise_type> h_;
};

// An awaitable that never suspends and yields a status code (operations the
// executor performed at once).
struct Ready {
    int rc;
    bool await_ready() const noexcept { return true; }
    void await_suspend(std::coroutine_handle<>) const noexcept {}
    int await_resume() const noexcept { return rc; }
};

}  // namespace expdg
