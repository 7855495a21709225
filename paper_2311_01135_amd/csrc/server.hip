// Continuous-batching SCF server: requests (molecules) arrive at any time,
// are admitted into resident batches while the HBM budget allows, every
// resident molecule advances one SCF iteration per progress() call, and
// converged molecules retire mid-flight (their results are copied out and a
// batch whose molecules have all retired releases its device memory).
//
// Overlap: each resident batch owns a HIP stream.  progress() first queues
// one iteration of every resident batch, then admits newcomers (host prep,
// one-electron integrals, grid, ERIs on their own stream) while those
// iterations run, then waits and retires.
//
// A molecule's arithmetic does not depend on which other molecules share its
// batch: the server fixes the per-molecule J/K and XC chunk counts (the
// batch heuristics would otherwise pick them from the batch size), so a
// result alone and in the mix differ only by the order of the J/K LDS atomic
// additions.
#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
#include <new>
#include <vector>

#include "kernels.h"

namespace {

using clk = std::chrono::steady_clock;

struct Request {
    long ticket;
    std::vector<int> Z;
    std::vector<double> xyz;
    int charge;
    size_t est_bytes;
};

struct Result {
    int state = 0;          // 0 queued, 1 resident, 2 done, 3 rejected
    double t_submit = 0.0, t_done = 0.0;
    double E = 0.0, homo = 0.0, lumo = 0.0, gap = 0.0;
    int status = 0, n_iter = 0, err = 0;
};

struct Resident {
    ks_batch* b = nullptr;
    hipStream_t stream = nullptr;
    std::vector<long> tickets;
    std::vector<char> reported;
    size_t bytes = 0;
    int n_active = 0;
    bool launched = false;
};

}  // namespace

struct ks_server {
    ks_options opt;
    size_t budget = 0;
    int max_batch = 64;
    std::deque<Request> queue;
    std::vector<Resident> res;
    std::vector<Result> results;
    size_t in_use = 0;
    long n_done = 0;
    bool wait_retire = false;   // an admission ran out of device memory: retry once a batch is released
    int fail_admissions = 0;    // testing hook: admissions that fail as if out of device memory
    clk::time_point t0;
};

using namespace ks;

static double now_s(const ks_server* s) { return std::chrono::duration<double>(clk::now() - s->t0).count(); }

// Device bytes a molecule will hold (ERIs of every unique quartet component,
// grid, matrices, DIIS history, work partials); used before admission.
static size_t estimate_bytes(const ks_options& o, int natom, int nbf)
{
    const double es = o.prec == KS_MIXED ? 4.0 : 8.0;
    const double npair = 0.5 * nbf * (nbf + 1.0);
    const double eri = 0.5 * npair * npair * 1.3 * es;
    const double grid = (double)natom * ((double)o.n_rad * o.n_theta * o.n_phi
                                         + (double)o.coarse_rad * o.coarse_theta * o.coarse_phi) * 32.0;
    const double np = std::ceil(nbf / 16.0) * 16.0;
    const double mats = (18.0 + 2.0 * o.diis_space) * nbf * nbf * 8.0;
    const double parts = (2.0 * 8.0 * np * np * 8.0) + 16.0 * np * np * es;
    return (size_t)(eri + grid + mats + parts) + (1u << 20);
}

static int validate(const int* Z, const double* xyz, int n, int charge, int basis, int* nbf)
{
    int ne = -charge, nb = 0;
    for (int a = 0; a < n; a++) {
        if (Z[a] != 1 && Z[a] != 6 && Z[a] != 7 && Z[a] != 8 && Z[a] != 9) return 0;
        if (basis == KS_BASIS_631G && Z[a] == 9) return 0;
        for (int k = 0; k < 3; k++)
            if (!std::isfinite(xyz[3 * a + k])) return 0;
        for (int c = 0; c < a; c++) {
            double d2 = 0.0;
            for (int k = 0; k < 3; k++) d2 += (xyz[3 * a + k] - xyz[3 * c + k]) * (xyz[3 * a + k] - xyz[3 * c + k]);
            if (std::sqrt(d2) / kBohrAng < 0.1) return 0;
        }
        ne += Z[a];
        nb += basis == KS_BASIS_631G ? (Z[a] == 1 ? 2 : 9) : (Z[a] == 1 ? 1 : 5);
    }
    *nbf = nb;
    return n > 0 && ne > 0 && !(ne & 1);
}

static void retire(ks_server* s, Resident& r)
{
    std::vector<MolState> st(r.tickets.size());
    if (hipMemcpyAsync(st.data(), r.b->d_state, sizeof(MolState) * st.size(), hipMemcpyDeviceToHost, r.stream) != hipSuccess ||
        hipStreamSynchronize(r.stream) != hipSuccess)
        return;
    for (size_t m = 0; m < r.tickets.size(); m++) {
        if (r.reported[m] || st[m].status == KS_MOL_ACTIVE) continue;
        Result& o = s->results[r.tickets[m]];
        if (ks_get_result(r.b, (int)m, &o.E, nullptr, nullptr, &o.homo, &o.lumo, &o.gap, &o.status, &o.n_iter) == KS_OK) {
            o.state = 2;
            o.t_done = now_s(s);
            r.reported[m] = 1;
            s->n_done++;
        }
    }
}

static void drop_resident(ks_server* s, size_t i)
{
    Resident& r = s->res[i];
    ks_batch_destroy(r.b);
    if (r.stream) (void)hipStreamDestroy(r.stream);
    s->in_use -= std::min(s->in_use, r.bytes);
    s->res.erase(s->res.begin() + i);
    s->wait_retire = false;
}

// Admit queued requests (at most cap) into one new batch while the budget
// allows.  The byte count per request is an estimate, so batch creation can
// still run out of device memory: then the requests stay queued and
// admission waits until a resident batch is released; with nothing resident
// the wave is retried with its first request alone, and only a single
// request that does not fit an empty device is rejected.
static ks_status admit(ks_server* s, int cap)
{
    if (s->queue.empty()) return KS_OK;
    if (s->wait_retire && !s->res.empty()) return KS_OK;
    size_t add = 0;
    int n = 0;
    for (const Request& q : s->queue) {
        if (n >= s->max_batch || n >= cap) break;
        if (s->in_use + add + q.est_bytes > s->budget && !(s->res.empty() && n == 0)) break;
        add += q.est_bytes;
        n++;
    }
    if (n == 0) return KS_OK;
    std::vector<int> na, Z;
    std::vector<double> xyz;
    std::vector<int> ch;
    Resident r;
    for (int i = 0; i < n; i++) {
        const Request& q = s->queue[i];
        na.push_back((int)q.Z.size());
        Z.insert(Z.end(), q.Z.begin(), q.Z.end());
        xyz.insert(xyz.end(), q.xyz.begin(), q.xyz.end());
        ch.push_back(q.charge);
        r.tickets.push_back(q.ticket);
    }
    KS_HIP(hipStreamCreateWithFlags(&r.stream, hipStreamNonBlocking));
    ks_status st;
    if (s->fail_admissions > 0) {
        s->fail_admissions--;
        set_error("admission failed: device memory (injected)");
        st = KS_ENOMEM;
    } else {
        st = ks_batch_create(&s->opt, n, na.data(), Z.data(), xyz.data(), ch.data(), r.stream, &r.b);
        if (st == KS_OK) st = ks_setup(r.b);
        if (st == KS_OK) st = eri_build(r.b);
    }
    if (st != KS_OK) {
        if (r.b) ks_batch_destroy(r.b);
        (void)hipStreamDestroy(r.stream);
        if (st == KS_ENOMEM) {
            if (!s->res.empty()) {
                s->wait_retire = true;        // the wave stays queued
                return KS_OK;
            }
            if (n > 1) return admit(s, 1);
            Result& o = s->results[s->queue.front().ticket];
            o.state = 3;
            o.err = st;
            o.t_done = now_s(s);
            s->queue.pop_front();
            return KS_OK;
        }
        // each request was validated at submit: this is a device failure,
        // and the whole admission wave is rejected
        for (int i = 0; i < n; i++) {
            Result& o = s->results[s->queue.front().ticket];
            o.state = 3;
            o.err = st;
            o.t_done = now_s(s);
            s->queue.pop_front();
        }
        return st;
    }
    for (int i = 0; i < n; i++) {
        s->results[s->queue.front().ticket].state = 1;
        s->queue.pop_front();
    }
    r.reported.assign(n, 0);
    r.bytes = batch_device_bytes(r.b);
    r.n_active = n;
    s->in_use += r.bytes;
    s->res.push_back(std::move(r));
    return KS_OK;
}

extern "C" {

ks_status ks_server_create(const ks_options* opt, size_t hbm_budget, int max_batch, ks_server** out)
{
    if (!out) {
        set_error("out is NULL");
        return KS_EINVAL;
    }
    *out = nullptr;
    ks_server* s = new (std::nothrow) ks_server();
    if (!s) {
        set_error("host allocation failed");
        return KS_ENOMEM;
    }
    ks_default_options(&s->opt);
    if (opt) s->opt = *opt;
    if (s->opt.jk_chunks <= 0) s->opt.jk_chunks = 8;
    if (s->opt.xc_chunks <= 0) s->opt.xc_chunks = 16;
    s->max_batch = max_batch > 0 ? max_batch : 64;
    if (hbm_budget == 0) {
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
            (void)hipGetLastError();
            set_error("hipMemGetInfo failed (no device?)");
            delete s;
            return KS_EDEVICE;
        }
        hbm_budget = fr / 10 * 8;
    }
    s->budget = hbm_budget;
    s->t0 = clk::now();
    *out = s;
    return KS_OK;
}

ks_status ks_server_submit(ks_server* s, int n_atoms, const int* Z, const double* xyz_angstrom, int charge, long* ticket)
{
    if (!s || !Z || !xyz_angstrom || !ticket) {
        set_error("NULL argument");
        return KS_EINVAL;
    }
    int nbf = 0;
    if (!validate(Z, xyz_angstrom, n_atoms, charge, s->opt.basis, &nbf)) {
        set_error("invalid molecule (element, coordinates, spacing or odd electron count)");
        return KS_EINVAL;
    }
    if (nbf > (s->opt.prec == KS_MIXED ? kMaxNbf : 82)) {
        set_error("%d basis functions exceeds the supported size", nbf);
        return KS_EUNSUPPORTED;
    }
    Request q;
    q.ticket = (long)s->results.size();
    q.Z.assign(Z, Z + n_atoms);
    q.xyz.assign(xyz_angstrom, xyz_angstrom + 3 * n_atoms);
    q.charge = charge;
    q.est_bytes = estimate_bytes(s->opt, n_atoms, nbf);
    Result o;
    o.t_submit = now_s(s);
    s->results.push_back(o);
    *ticket = q.ticket;
    s->queue.push_back(std::move(q));
    return KS_OK;
}

ks_status ks_server_progress(ks_server* s, int* n_finished)
{
    if (!s) {
        set_error("server handle is NULL");
        return KS_EINVAL;
    }
    const long before = s->n_done;
    ks_status st;
    // 1. one iteration of every resident batch, each on its own stream
    for (Resident& r : s->res) {
        r.launched = false;
        if (r.n_active > 0) {
            if ((st = step_launch(r.b))) return st;
            r.launched = true;
        }
    }
    // 2. admit newcomers while those iterations run
    if ((st = admit(s, s->max_batch))) return st;
    // 3. wait, retire converged molecules, release empty batches
    for (Resident& r : s->res) {
        if (!r.launched) continue;
        if ((st = step_finish(r.b, &r.n_active))) return st;
        retire(s, r);
    }
    for (size_t i = s->res.size(); i-- > 0;)
        if (s->res[i].n_active == 0 && s->res[i].launched) drop_resident(s, i);
    if (n_finished) *n_finished = (int)(s->n_done - before);
    return KS_OK;
}

ks_status ks_server_poll(const ks_server* s, long ticket, double* E, double* homo, double* lumo, double* gap,
                         int* status, int* n_iter, double* latency_s)
{
    if (!s || ticket < 0 || ticket >= (long)s->results.size()) {
        set_error("unknown ticket");
        return KS_EINVAL;
    }
    const Result& o = s->results[ticket];
    if (o.state == 3) {
        set_error("request rejected at admission (status %d)", o.err);
        return (ks_status)o.err;
    }
    if (o.state != 2) return KS_ESTATE;
    if (E) *E = o.E;
    if (homo) *homo = o.homo;
    if (lumo) *lumo = o.lumo;
    if (gap) *gap = o.gap;
    if (status) *status = o.status;
    if (n_iter) *n_iter = o.n_iter;
    if (latency_s) *latency_s = o.t_done - o.t_submit;
    return KS_OK;
}

ks_status ks_server_stats(const ks_server* s, int* queued, int* resident, long* done, size_t* bytes_in_use)
{
    if (!s) {
        set_error("server handle is NULL");
        return KS_EINVAL;
    }
    int nres = 0;
    for (const Resident& r : s->res) nres += r.n_active;
    if (queued) *queued = (int)s->queue.size();
    if (resident) *resident = nres;
    if (done) *done = s->n_done;
    if (bytes_in_use) *bytes_in_use = s->in_use;
    return KS_OK;
}

ks_status ks_server_fail_admissions(ks_server* s, int n)
{
    if (!s || n < 0) {
        set_error("server handle is NULL or count negative");
        return KS_EINVAL;
    }
    s->fail_admissions = n;
    return KS_OK;
}

void ks_server_destroy(ks_server* s)
{
    if (!s) return;
    while (!s->res.empty()) drop_resident(s, s->res.size() - 1);
    delete s;
}

}  // extern "C"
