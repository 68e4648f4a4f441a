// GRAPE-5-compatible host interface (Sec. 3.6): host double arrays of
// 3-vectors, converted to and from the FP32 structure-of-arrays device
// layout of the pgh calls.  Host code only; the force work runs in the
// library's kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>
#include <vector>

#include "grape5.h"

namespace {

struct G5State {
    pgh_ctx *ctx = nullptr;
    bool table = false;
    int n = 0;  // g5_set_n, applied when forces are computed (it may precede g5_set_xmj)
    // device staging, FP32 structure of arrays
    float *dj = nullptr;  // 4 x jcap: x, y, z, m
    size_t jcap = 0;
    float *di = nullptr;  // 7 x icap: x, y, z, ax, ay, az, phi
    size_t icap = 0;
    std::vector<float> host;  // conversion buffer
    std::string err;
    bool failed = false;
};

G5State g5;

void set_error(const std::string &m)
{
    g5.err = m;
    g5.failed = true;
}

bool check(int status, const char *what)
{
    if (status == PGH_OK) return true;
    const char *m = pgh_last_error(g5.ctx);
    set_error(std::string(what) + ": " + (m ? m : "error"));
    return false;
}

bool ensure(float **buf, size_t *cap, size_t per, size_t n)
{
    if (n <= *cap) return true;
    size_t want = std::max(n, *cap * 2);
    float *p = nullptr;
    if (hipMalloc((void **)&p, per * want * sizeof(float)) != hipSuccess) {
        set_error("hipMalloc of the staging arrays failed");
        return false;
    }
    (void)hipDeviceSynchronize();
    (void)hipFree(*buf);
    *buf = p;
    *cap = want;
    return true;
}

double trampoline(double r, void *user)
{
    return reinterpret_cast<double (*)(double)>(user)(r);
}

bool opened()
{
    if (g5.ctx) return true;
    set_error("g5_open has not been called");
    return false;
}

}  // namespace

extern "C" {

void g5_open(void)
{
    g5.failed = false;
    if (g5.ctx) return;
    pgh_ctx *c = nullptr;
    if (pgh_open(&c, 0, nullptr) != PGH_OK) {
        const char *m = pgh_last_error(nullptr);
        set_error(std::string("pgh_open: ") + (m ? m : "error"));
        return;
    }
    g5.ctx = c;
    g5.table = false;
}

void g5_close(void)
{
    g5.failed = false;
    if (!g5.ctx) return;
    (void)pgh_close(g5.ctx);
    (void)hipFree(g5.dj);
    (void)hipFree(g5.di);
    g5 = G5State{};
}

void g5_set_eps_to_all(double eps)
{
    g5.failed = false;
    if (opened()) check(pgh_set_eps_to_all(g5.ctx, (float)eps), "g5_set_eps_to_all");
}

void g5_set_n(int nj)
{
    g5.failed = false;
    if (!opened()) return;
    if (nj < 0) return set_error("g5_set_n: negative nj");
    g5.n = nj;
}

void g5_set_xmj(int adr, int nj, double (*xj)[3], double *mj)
{
    g5.failed = false;
    if (!opened()) return;
    if (adr < 0 || nj < 0) return set_error("g5_set_xmj: negative adr or nj");
    if (nj == 0) return;
    if (!xj || !mj) return set_error("g5_set_xmj: NULL array");
    const size_t n = (size_t)nj;
    if (!ensure(&g5.dj, &g5.jcap, 4, n)) return;
    g5.host.resize(4 * n);
    for (size_t k = 0; k < n; ++k) {
        g5.host[k] = (float)xj[k][0];
        g5.host[n + k] = (float)xj[k][1];
        g5.host[2 * n + k] = (float)xj[k][2];
        g5.host[3 * n + k] = (float)mj[k];
    }
    for (int a = 0; a < 4; ++a)
        if (hipMemcpy(g5.dj + a * g5.jcap, g5.host.data() + a * n, n * sizeof(float),
                      hipMemcpyHostToDevice) != hipSuccess)
            return set_error("g5_set_xmj: copy to the device failed");
    const float *d = g5.dj;
    if (!check(pgh_set_xmj(g5.ctx, adr, nj, d, d + g5.jcap, d + 2 * g5.jcap, d + 3 * g5.jcap),
               "g5_set_xmj"))
        return;
    if (hipDeviceSynchronize() != hipSuccess) set_error("g5_set_xmj: device error");
}

void g5_calculate_force_on_x(double (*xi)[3], double (*ai)[3], double *pi, int ni)
{
    g5.failed = false;
    if (!opened()) return;
    if (ni < 0) return set_error("g5_calculate_force_on_x: negative ni");
    if (ni == 0) return;
    if (!xi || !ai) return set_error("g5_calculate_force_on_x: NULL array");
    const size_t n = (size_t)ni;
    if (!ensure(&g5.di, &g5.icap, 7, n)) return;
    g5.host.resize(7 * n);
    for (size_t k = 0; k < n; ++k) {
        g5.host[k] = (float)xi[k][0];
        g5.host[n + k] = (float)xi[k][1];
        g5.host[2 * n + k] = (float)xi[k][2];
    }
    float *d = g5.di;
    const size_t cap = g5.icap;
    for (int a = 0; a < 3; ++a)
        if (hipMemcpy(d + a * cap, g5.host.data() + a * n, n * sizeof(float),
                      hipMemcpyHostToDevice) != hipSuccess)
            return set_error("g5_calculate_force_on_x: copy to the device failed");
    if (!check(pgh_set_n(g5.ctx, g5.n), "g5_calculate_force_on_x (the count of g5_set_n)")) return;
    int st;
    if (g5.table)
        st = pgh_calc_table(g5.ctx, ni, d, d + cap, d + 2 * cap, d + 3 * cap, d + 4 * cap,
                            d + 5 * cap, nullptr);
    else
        st = pgh_calc_newton(g5.ctx, ni, d, d + cap, d + 2 * cap, nullptr, d + 3 * cap,
                             d + 4 * cap, d + 5 * cap, pi ? d + 6 * cap : nullptr);
    if (!check(st, "g5_calculate_force_on_x")) return;
    const int outs = (!g5.table && pi) ? 4 : 3;
    for (int a = 0; a < outs; ++a)
        if (hipMemcpy(g5.host.data() + (3 + a) * n, d + (3 + a) * cap, n * sizeof(float),
                      hipMemcpyDeviceToHost) != hipSuccess)
            return set_error("g5_calculate_force_on_x: copy from the device failed");
    for (size_t k = 0; k < n; ++k) {
        ai[k][0] = g5.host[3 * n + k];
        ai[k][1] = g5.host[4 * n + k];
        ai[k][2] = g5.host[5 * n + k];
        if (pi) pi[k] = g5.table ? 0.0 : (double)g5.host[6 * n + k];
    }
}

int g5_set_force_table(int E, int F, double rcut, double (*f_over_r)(double r))
{
    g5.failed = false;
    if (!opened()) return PGH_ESTATE;
    if (!f_over_r) {
        set_error("g5_set_force_table: NULL function");
        return PGH_EINVAL;
    }
    const int st = pgh_build_table(g5.ctx, E, F, (float)rcut, trampoline,
                                   reinterpret_cast<void *>(f_over_r), nullptr);
    if (!check(st, "g5_set_force_table")) return st;
    g5.table = true;
    return PGH_OK;
}

void g5_use_newton(void)
{
    g5.failed = false;
    g5.table = false;
}

const char *g5_last_error(void) { return g5.failed ? g5.err.c_str() : nullptr; }

}  // extern "C"
