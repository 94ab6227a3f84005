/*
 * Test-process aid: on SIGSEGV, SIGBUS or SIGABRT print the native call stack (library and
 * offset of every frame) to stderr, then hand the signal to the handler that was installed
 * before (Python's faulthandler, which adds the Python stack).  Loaded by tests/conftest.py
 * when built; compiled by __graft_entry__.build().
 */
#include <execinfo.h>
#include <signal.h>
#include <string.h>
#include <unistd.h>

static struct sigaction g_prev[3];
static const int g_sigs[3] = {SIGSEGV, SIGBUS, SIGABRT};

static void on_signal(int sig, siginfo_t* info, void* ctx) {
    (void)info;
    (void)ctx;
    static const char head[] = "\n---- native backtrace ----\n";
    void* frames[64];
    ssize_t w = write(2, head, sizeof head - 1);
    (void)w;
    int n = backtrace(frames, 64);
    backtrace_symbols_fd(frames, n, 2);
    for (int i = 0; i < 3; ++i)
        if (g_sigs[i] == sig) sigaction(sig, &g_prev[i], NULL);
    raise(sig); /* delivered to the previous handler once this one returns */
}

int native_backtrace_install(void) {
    void* warm[2];
    backtrace(warm, 2); /* loads the unwinder now, not inside the handler */
    struct sigaction sa;
    memset(&sa, 0, sizeof sa);
    sa.sa_sigaction = on_signal;
    sa.sa_flags = SA_SIGINFO | SA_ONSTACK;
    sigemptyset(&sa.sa_mask);
    for (int i = 0; i < 3; ++i)
        if (sigaction(g_sigs[i], &sa, &g_prev[i]) != 0) return -1;
    return 0;
}
