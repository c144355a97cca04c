/* Test infrastructure: on SIGSEGV / SIGBUS / SIGABRT print the faulting
 * address and a native backtrace to stderr (frames in shared libraries as
 * library+offset), then hand the signal to the handler that was installed
 * before (Python's faulthandler under pytest).  Loaded by tests/conftest.py
 * when AMGDD_CRASH_TRACE=1.  Build: gcc -O1 -shared -fPIC crash_trace.c -o crash_trace.so */
#define _GNU_SOURCE
#include <execinfo.h>
#include <signal.h>
#include <stdio.h>
#include <string.h>
#include <unistd.h>

static struct sigaction prev[3];
static const int sigs[3] = {SIGSEGV, SIGBUS, SIGABRT};

static void handler(int sig, siginfo_t *si, void *uc) {
  char msg[160];
  int n = snprintf(msg, sizeof msg, "[crash_trace] signal %d (%s), address %p, thread %ld; native backtrace:\n", sig,
                   strsignal(sig), si ? si->si_addr : 0, (long)gettid());
  if (n > 0) (void)!write(2, msg, (size_t)n);
  void *bt[96];
  int k = backtrace(bt, 96);
  backtrace_symbols_fd(bt, k, 2);
  for (int i = 0; i < 3; ++i)
    if (sigs[i] == sig) {
      struct sigaction *p = &prev[i];
      if ((p->sa_flags & SA_SIGINFO) && p->sa_sigaction) {
        p->sa_sigaction(sig, si, uc);
        return;
      }
      if (p->sa_handler != SIG_DFL && p->sa_handler != SIG_IGN) {
        p->sa_handler(sig);
        return;
      }
      sigaction(sig, p, 0);
      raise(sig);
      return;
    }
}

int crash_trace_install(void) {
  void *warm[2];
  backtrace(warm, 2); /* load libgcc's unwinder now, not inside the handler */
  for (int i = 0; i < 3; ++i) {
    struct sigaction sa;
    memset(&sa, 0, sizeof sa);
    sa.sa_sigaction = handler;
    sa.sa_flags = SA_SIGINFO | SA_ONSTACK;
    sigemptyset(&sa.sa_mask);
    if (sigaction(sigs[i], &sa, &prev[i]) != 0) return -1;
  }
  return 0;
}
