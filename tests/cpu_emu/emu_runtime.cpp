// Fiber runtime of the test-only CPU build of the kernels (x86-64 SysV).
#include <sanitizer/common_interface_defs.h>

// Fiber annotations for AddressSanitizer; weak, so that the build without the
// sanitizer (a shared library for numerical checks) links and skips them.
extern "C" {
__attribute__((weak)) void __sanitizer_start_switch_fiber(void**, const void*, size_t);
__attribute__((weak)) void __sanitizer_finish_switch_fiber(void*, const void**, size_t*);
}
#define ASAN_START(a, b, c) \
  do { if (&__sanitizer_start_switch_fiber) __sanitizer_start_switch_fiber(a, b, c); } while (0)
#define ASAN_FINISH(a, b, c) \
  do { if (&__sanitizer_finish_switch_fiber) __sanitizer_finish_switch_fiber(a, b, c); } while (0)

#include "hip/hip_runtime.h"

thread_local uint3 threadIdx;
thread_local uint3 blockIdx;
thread_local dim3 blockDim;
thread_local dim3 gridDim;

extern "C" void lrdm_emu_switch(void** save_sp, void* load_sp);
asm(R"(
.text
.globl lrdm_emu_switch
.type lrdm_emu_switch,@function
lrdm_emu_switch:
  pushq %rbp
  pushq %rbx
  pushq %r12
  pushq %r13
  pushq %r14
  pushq %r15
  movq %rsp, (%rdi)
  movq %rsi, %rsp
  popq %r15
  popq %r14
  popq %r13
  popq %r12
  popq %rbx
  popq %rbp
  ret
.size lrdm_emu_switch, .-lrdm_emu_switch
)");

namespace lrdm_emu {

thread_local Block* cur = nullptr;
thread_local Fiber* cur_fiber = nullptr;
thread_local int tid_linear = 0;

namespace {
constexpr size_t kStack = 256 * 1024;
struct StackPool {
  std::vector<char*> stacks;
  ~StackPool() {
    for (char* p : stacks) std::free(p);
  }
};
thread_local StackPool pool;

void to_scheduler() {
  void* fake = nullptr;
  ASAN_START(&fake, cur->sched_stack_bottom, cur->sched_stack_size);
  lrdm_emu_switch(&cur_fiber->sp, cur->sched_sp);
  ASAN_FINISH(fake, nullptr, nullptr);
}

[[noreturn]] void fiber_entry() {
  ASAN_FINISH(nullptr, nullptr, nullptr);
  cur->body();
  cur_fiber->done = true;
  ASAN_START(nullptr, cur->sched_stack_bottom, cur->sched_stack_size);
  lrdm_emu_switch(&cur_fiber->sp, cur->sched_sp);
  std::abort();
}

void resume(Block& b, Fiber& f) {
  cur_fiber = &f;
  tid_linear = f.tid;
  threadIdx = f.idx;
  void* fake = nullptr;
  ASAN_START(&fake, f.stack, kStack);
  lrdm_emu_switch(&b.sched_sp, f.sp);
  ASAN_FINISH(fake, &b.sched_stack_bottom, &b.sched_stack_size);
}
}  // namespace

Block& worker_block() {
  static thread_local Block b;
  return b;
}

void yield_wait(int kind) {
  cur_fiber->wait = kind;
  to_scheduler();
}

void run_block(Block& b, dim3 block, uint3, size_t smem) {
  const int nt = (int)(block.x * block.y * block.z);
  b.nthreads = nt;
  b.fibers.assign(nt, Fiber{});
  if ((int)b.xch.size() < (nt + 63) / 64) b.xch.resize((nt + 63) / 64, std::vector<double>(64 * 32, 0.0));
  // exactly the requested dynamic LDS, so that AddressSanitizer sees any access
  // past its end
  b.dyn = std::vector<unsigned char>(smem ? smem : 1, (unsigned char)0xAB);
  while ((int)pool.stacks.size() < nt) pool.stacks.push_back(static_cast<char*>(std::malloc(kStack)));
  cur = &b;
  for (int t = 0; t < nt; ++t) {
    Fiber& f = b.fibers[t];
    f.tid = t;
    f.idx = uint3{(unsigned)(t % block.x), (unsigned)((t / block.x) % block.y),
                  (unsigned)(t / (block.x * block.y))};
    f.stack = pool.stacks[t];
    // initial frame: six callee-saved registers, then the entry as return address;
    // rsp at entry is 8 mod 16 as after a call.
    uintptr_t top = (reinterpret_cast<uintptr_t>(f.stack) + kStack) & ~uintptr_t(15);
    void** sp = reinterpret_cast<void**>(top);
    *--sp = nullptr;                                   // padding
    *--sp = reinterpret_cast<void*>(&fiber_entry);     // return address
    for (int r = 0; r < 6; ++r) *--sp = nullptr;      // rbp rbx r12 r13 r14 r15
    f.sp = sp;
  }
  const int nw = (nt + 63) / 64;
  for (;;) {
    bool ran = false;
    for (int t = 0; t < nt; ++t) {
      Fiber& f = b.fibers[t];
      if (!f.done && f.wait == 0) {
        resume(b, f);
        ran = true;
      }
    }
    // release wavefront barriers whose live lanes all arrived
    bool released = false;
    for (int w = 0; w < nw; ++w) {
      bool all = true, any = false;
      for (int t = 64 * w; t < std::min(nt, 64 * w + 64); ++t) {
        const Fiber& f = b.fibers[t];
        if (f.done) continue;
        any = true;
        if (f.wait != 2) all = false;
      }
      if (any && all) {
        for (int t = 64 * w; t < std::min(nt, 64 * w + 64); ++t) b.fibers[t].wait = 0;
        released = true;
      }
    }
    // release the block barrier when every live thread waits on it
    bool all_block = true, live = false;
    for (const Fiber& f : b.fibers) {
      if (f.done) continue;
      live = true;
      if (f.wait != 1) all_block = false;
    }
    if (!live) break;
    if (all_block) {
      for (Fiber& f : b.fibers) f.wait = 0;
      released = true;
    }
    if (!ran && !released) {
      std::fprintf(stderr, "emulation deadlock: block barrier and wavefront barrier mixed\n");
      std::abort();
    }
  }
  cur = nullptr;
}

// Persistent pool of host threads that run the blocks of each launch; each
// keeps its fiber stacks between launches.
namespace {
struct Pool {
  std::mutex m;
  std::condition_variable cv_job, cv_done;
  const std::function<void(uint3)>* fn = nullptr;
  dim3 grid;
  long total = 0;
  std::atomic<long> next{0};
  int active = 0;
  long generation = 0;
  bool stop = false;
  std::vector<std::thread> workers;

  explicit Pool(int n) {
    for (int w = 0; w < n; ++w) workers.emplace_back([this] { loop(); });
  }
  ~Pool() {
    {
      std::lock_guard<std::mutex> lk(m);
      stop = true;
    }
    cv_job.notify_all();
    for (auto& t : workers) t.join();
  }
  void loop() {
    long seen = 0;
    for (;;) {
      {
        std::unique_lock<std::mutex> lk(m);
        cv_job.wait(lk, [&] { return stop || generation != seen; });
        if (stop) return;
        seen = generation;
      }
      for (;;) {
        const long i = next.fetch_add(1);
        if (i >= total) break;
        const unsigned bx = (unsigned)(i % grid.x), by = (unsigned)((i / grid.x) % grid.y),
                       bz = (unsigned)(i / ((long)grid.x * grid.y));
        (*fn)(uint3{bx, by, bz});
      }
      std::lock_guard<std::mutex> lk(m);
      if (--active == 0) cv_done.notify_all();
    }
  }
  void run(dim3 g, const std::function<void(uint3)>& f) {
    std::unique_lock<std::mutex> lk(m);
    fn = &f;
    grid = g;
    total = (long)g.x * g.y * g.z;
    next = 0;
    active = (int)workers.size();
    ++generation;
    cv_job.notify_all();
    cv_done.wait(lk, [&] { return active == 0; });
  }
};
}  // namespace

void parallel_blocks(dim3 grid, const std::function<void(uint3)>& fn) {
  static Pool pool(8);
  pool.run(grid, fn);
}

}  // namespace lrdm_emu
