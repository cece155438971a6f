// Host side of libsht: plan construction (ring geometry, FFT plans, Legendre seed
// tables, work lists, workspace) and the C ABI declared in include/sht.h.
#include "../../include/sht.h"
#include "fft_internal.h"

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

using namespace sht;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg)
{
    g_err = msg;
    return code;
}

#define HIPCHK(expr)                                                                         \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess) {                                                              \
            int c_ = (e_ == hipErrorOutOfMemory) ? SHT_ERR_NOMEM : SHT_ERR_DEVICE;           \
            return fail(c_, std::string(#expr) + ": " + hipGetErrorString(e_));               \
        }                                                                                    \
    } while (0)

typedef long double ld;
const ld PI_L = 3.141592653589793238462643383279502884197L;

// Static workspace of sht_alm2map_noalloc: a device array each GPU holds from
// the first use of the library on it until the process ends.  Host code never
// passes the array's name to a kernel (on the host it only names the symbol):
// plan creation resolves its device address once per device with
// hipGetSymbolAddress, and that address is what the kernels receive.
constexpr size_t SCRATCH_BYTES = (size_t)256 << 20;
static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[MAX_DEVICES] = {};

// The device address of `scratch` on the current device (resolved once per device).
int resolve_scratch(int dev, void** out)
{
    if (dev < 0 || dev >= MAX_DEVICES) return fail(SHT_ERR_UNSUPPORTED, "device index beyond the static workspace table");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(SHT_ERR_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return SHT_OK;
}

// Device allocation that records its size (for the table accounting).
struct Dev {
    void* p = nullptr;
    size_t n = 0;
};

struct SeedSet {
    int spin = -1;
    Dev mu, kk, seedoff, lsig, tileoff, ftileoff, rowoff, coef;
    int64_t stride = 0;  // seeds per SoA array
    int ntiles = 0;      // l tiles of TL over all m
    int64_t rows = 0;    // m-major coefficient rows over all m
};

}  // namespace

struct sht_plan_s {
    int device = 0;
    int nside = 0, lmax = 0, spin = 0, ncomp = 1, cap = 0, nmaps = 0, chunk = 0, prec = SHT_FP64;
    int nring = 0, rn = 0, nrc = 0;
    int64_t npix = 0;
    hipStream_t stream = nullptr;

    std::vector<RingDev> rings;
    std::vector<FftLen> lens;
    std::vector<Dev> owned;  // all table allocations
    RingDev* d_rings = nullptr;
    FftLen* d_lens = nullptr;
    double2* d_tw = nullptr;
    double2* d_bhat = nullptr;
    SeedSet s0, s2;

    // FFT work items for the current chunk size
    // FFT work lists per chunk width (map pairs per chunk), kept so that changing
    // the chunk between calls (serving batches of different sizes) reuploads nothing
    struct ItemSet {
        Dev dev;
        std::vector<FftClass> classes;
    };
    std::map<int, ItemSet> item_sets;
    std::vector<FftClass> classes;  // the current width's classes
    int items_npairs = -1;
    int64_t ldx_cur = 0;            // row pitch of the m-major arrays for the chunk being run
    int nm_cur = 0;                 // map sets of the chunk being run

    // workspace
    void* ws = nullptr;
    size_t ws_bytes = 0;
    bool ws_owned = false;
    // iteration buffers (data spectra, residual norms), plan owned, lazily allocated
    double* F = nullptr;
    size_t F_bytes = 0;
    double* norms = nullptr;
    size_t table_bytes = 0;
    double* R = nullptr;  // immediate iteration: residual spectra, bin-major (lazily)
    size_t R_bytes = 0;

    // ring skip bound per m (first ring chunk where either spin's Legendre values
    // of m are significant), and the immediate-iteration schedule built from it
    std::vector<int> cmin;
    struct Levels {
        bool built = false;
        std::vector<int> start, len;           // per level: first entry in mlist, entries
        std::vector<int> ntiles0, ntiles2;     // per level: l tiles of the listed m per spin
        Dev mlist, pref0, pref2, cmin;         // device: m per entry; per-level tile prefix sums
    } lev;

    // device address of the static workspace on the plan's device
    void* scratch = nullptr;

    // part `part` of `nparts` of the orders m (sht_plan_create_part): own[m] = 1 for
    // the m this plan transforms; d_own its device copy, d_mlist the owned m
    int part = 0, nparts = 1, nown = 0;
    std::vector<unsigned char> own;
    Dev d_own, d_mlist;

    // optional per-stage profiling
    bool profiling = false;
    struct Rec { int stage; hipEvent_t a, b; };
    std::vector<Rec> recs;
};

namespace {

// Brackets the launches of one stage with HIP events when profiling is on.
struct StageTimer {
    sht_plan p;
    int stage;
    hipEvent_t a = nullptr, b = nullptr;
    StageTimer(sht_plan p_, int stage_) : p(p_), stage(stage_)
    {
        if (!p->profiling) return;
        if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) { a = b = nullptr; return; }
        (void)hipEventRecord(a, p->stream);
    }
    ~StageTimer()
    {
        if (!a) return;
        (void)hipEventRecord(b, p->stream);
        p->recs.push_back(sht_plan_s::Rec{stage, a, b});
    }
};

// whether the plan transforms order m: pairs (q, lmax - q) of the folded order
// 0, lmax, 1, lmax - 1, ... are dealt to the parts in turn, q mod nparts
bool owns(sht_plan p, int m) { return p->nparts <= 1 || p->own[m]; }

int dev_alloc(sht_plan p, Dev& d, size_t bytes)
{
    d.n = bytes;
    if (bytes == 0) { d.p = nullptr; return SHT_OK; }
    hipError_t e = hipMalloc(&d.p, bytes);
    if (e != hipSuccess) {
        d.p = nullptr;
        return fail(SHT_ERR_NOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed: " + hipGetErrorString(e));
    }
    p->owned.push_back(d);
    p->table_bytes += bytes;
    return SHT_OK;
}

template <typename T>
int upload(sht_plan p, Dev& d, const std::vector<T>& v)
{
    int rc = dev_alloc(p, d, v.size() * sizeof(T));
    if (rc) return rc;
    if (!v.empty()) HIPCHK(hipMemcpy(d.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
    return SHT_OK;
}

// --------------------------------------------------------------------------
// HEALPix RING geometry (Gorski et al. 2005): ring i = 1 .. 4 nside - 1
// --------------------------------------------------------------------------
void build_rings(sht_plan p)
{
    const int64_t ns = p->nside;
    p->nring = 4 * p->nside - 1;
    p->rn = 2 * p->nside;  // northern rings including the equator
    p->npix = 12 * ns * ns;
    p->rings.resize(p->nring);
    for (int64_t i = 1; i <= 4 * ns - 1; ++i) {
        RingDev r{};
        ld z, sth;
        if (i < ns || i > 3 * ns) {
            int64_t j = (i < ns) ? i : 4 * ns - i;
            ld onemz = (ld)(j * j) / (3.0L * (ld)ns * (ld)ns);
            z = 1.0L - onemz;
            r.omz = (double)onemz;
            sth = sqrtl(onemz * (2.0L - onemz));
            r.n = (int)(4 * j);
            r.s = 1;
            if (i < ns) r.first = 2 * j * (j - 1);
            else { r.first = p->npix - 2 * j * (j + 1); z = -z; }
        } else {
            z = (ld)(4 * ns - 2 * i) / (3.0L * (ld)ns);
            sth = sqrtl((1.0L - z) * (1.0L + z));
            const int64_t az = (4 * ns - 2 * i) < 0 ? -(4 * ns - 2 * i) : (4 * ns - 2 * i);
            r.omz = (double)((ld)(3 * ns - az) / (3.0L * (ld)ns));
            r.n = (int)(4 * ns);
            r.s = ((i - ns) % 2 == 0) ? 1 : 0;
            r.first = 2 * ns * (ns - 1) + (i - ns) * 4 * ns;
        }
        r.z = (double)z;
        r.sth = (double)sth;
        r.mcut = p->lmax;  // narrowed by build_mcut once the skip tables exist
        p->rings[i - 1] = r;
    }
}

// --------------------------------------------------------------------------
// FFT plans
// --------------------------------------------------------------------------
bool factor_radices(int n, std::vector<int>& rad)
{
    rad.clear();
    int t = n;
    while (t % 4 == 0) { rad.push_back(4); t /= 4; }
    while (t % 2 == 0) { rad.push_back(2); t /= 2; }
    for (int q : {3, 5, 7})
        while (t % q == 0) { rad.push_back(q); t /= q; }
    return t == 1;
}

int smooth_at_least(int x)
{
    for (int m = x;; ++m) {
        int t = m;
        for (int q : {2, 3, 5, 7})
            while (t % q == 0) t /= q;
        if (t == 1) return m;
    }
}

void push_twiddles(std::vector<double2>& pool, int n)
{
    // e^{-i pi j / n}, j = 0 .. 2n-1, from long-double sin/cos of the exact angle
    for (int j = 0; j < 2 * n; ++j) {
        ld ang = PI_L * (ld)j / (ld)n;
        pool.push_back(make_double2((double)cosl(ang), (double)(-sinl(ang))));
    }
}

int build_fft(sht_plan p)
{
    std::map<int, int> len_index;
    std::map<int, int64_t> tw_of;  // length -> twiddle offset
    std::vector<double2> pool;
    std::vector<int> blue;
    int64_t bhat_total = 0;
    int max_blue_m = 0;
    for (auto& r : p->rings) {
        auto it = len_index.find(r.n);
        if (it != len_index.end()) { r.len = it->second; continue; }
        FftLen L{};
        L.n = r.n;
        std::vector<int> rad;
        bool direct = factor_radices(r.n, rad);
        if (!tw_of.count(r.n)) { tw_of[r.n] = (int64_t)pool.size(); push_twiddles(pool, r.n); }
        L.tw = tw_of[r.n];
        int len = r.n;
        if (!direct) {
            L.blue = 1;
            // chirp e^{-i pi j^2 / n}: the angle is reduced exactly (j^2 mod 2n) before the long-double sincos
            L.chirp = (int64_t)pool.size();
            for (int j = 0; j < r.n; ++j) {
                const int64_t q = ((int64_t)j * j) % (2 * (int64_t)r.n);
                const ld ang = PI_L * (ld)q / (ld)r.n;
                pool.push_back(make_double2((double)cosl(ang), (double)(-sinl(ang))));
            }
            // convolution length: a power of two up to 2^12 (compile-time
            // kernels of k_fft_p2.hip), else the smallest 7-smooth length
            int pm = 64, lg = 6;
            while (pm < 2 * r.n - 1) { pm *= 2; ++lg; }
            if (lg <= 12 && p2_seqs_per_group(lg) > 0) {
                L.m = pm;
                L.bp2 = lg;
            } else {
                L.m = smooth_at_least(2 * r.n - 1);
            }
            if (L.m > 16 * FFT_THREADS && r.n <= 16 * FFT_THREADS) {
                // the convolution would not fit the LDS: n = 4j runs as four
                // Bluestein DFTs of length j through 4096 points and a radix-4
                // step, one map pair per workgroup (k_fft_four.hip); the length-j
                // Bluestein data sit in an entry of their own
                const int j = r.n / 4;
                if (r.n % 4 || 2 * j - 1 > 4096) return fail(SHT_ERR_UNSUPPORTED, "ring FFT length beyond the four-step plan");
                FftLen J{};
                J.n = j;
                J.blue = 1;
                J.m = 4096;
                J.bp2 = 12;
                J.chirp = (int64_t)pool.size();
                for (int s = 0; s < j; ++s) {
                    const int64_t q = ((int64_t)s * s) % (2 * (int64_t)j);
                    const ld ang = PI_L * (ld)q / (ld)j;
                    pool.push_back(make_double2((double)cosl(ang), (double)(-sinl(ang))));
                }
                std::vector<int> radm;
                factor_radices(J.m, radm);
                J.nstage = (int)radm.size();
                for (size_t q = 0; q < radm.size(); ++q) J.radix[q] = radm[q];
                if (!tw_of.count(J.m)) { tw_of[J.m] = (int64_t)pool.size(); push_twiddles(pool, J.m); }
                J.tw = J.twm = tw_of[J.m];
                J.bhat = bhat_total;
                bhat_total += J.m;
                J.nseq = 1;
                J.ldsc = J.m;
                J.lstride = J.m + J.m / 16;
                J.lds = J.lstride;
                max_blue_m = std::max(max_blue_m, J.m);
                L.sub = (int)p->lens.size();
                blue.push_back(L.sub);
                p->lens.push_back(J);
                L.blue = 0;
                L.four = 1;
                L.m = 0;
                L.bp2 = 0;
                L.nstage = 0;
                L.nseq = 1;
                L.lgseq = 0;
                L.ldsc = r.n;
                L.lstride = r.n;
                L.lds = r.n;
                r.len = (int)p->lens.size();
                len_index[r.n] = r.len;
                p->lens.push_back(L);
                continue;
            }
            factor_radices(L.m, rad);
            if (!tw_of.count(L.m)) { tw_of[L.m] = (int64_t)pool.size(); push_twiddles(pool, L.m); }
            L.twm = tw_of[L.m];
            L.bhat = bhat_total;
            bhat_total += L.m;
            len = L.m;
            max_blue_m = std::max(max_blue_m, L.m);
        }
        if ((int)rad.size() > MAX_STAGES) return fail(SHT_ERR_UNSUPPORTED, "ring FFT needs too many stages");
        L.nstage = (int)rad.size();
        for (size_t k = 0; k < rad.size(); ++k) L.radix[k] = rad[k];
        if (len > 16 * FFT_THREADS) return fail(SHT_ERR_UNSUPPORTED, "ring FFT length beyond the LDS plan");
        // map pairs per workgroup: fill up to 1024 complex values when small, else 4096
        int cap = (len <= 1024) ? 1024 : (len <= 4096 ? 4096 : 8192);
        L.lgseq = 0;
        while (L.lgseq < 4 && (2 << L.lgseq) * len <= cap) ++L.lgseq;
        L.nseq = 1 << L.lgseq;
        L.ldsc = L.nseq * len;
        // padded sequence stride, congruent to 16/nseq complex values modulo 16, so
        // that the nseq sequences interleaved across a wave start on distinct banks
        {
            const int base = len + len / 16, want = (16 / L.nseq) % 16;
            L.lstride = base + (((want - base) % 16) + 16) % 16;
        }
        L.lds = L.nseq * L.lstride;
        // power-of-two lengths run the compile-time-length kernels, which fix
        // their own map pairs per workgroup (the runtime-length layout above is
        // kept for the residual kernel of the iteration)
        L.p2 = 0;
        if (L.bp2) {
            const int S = p2_seqs_per_group(L.bp2);
            L.nseq = S;
            L.lgseq = 0;
            while ((1 << L.lgseq) < S) ++L.lgseq;
            L.ldsc = S * L.m;
            const int base = len + len / 16, want = (16 / L.nseq) % 16;
            L.lstride = base + (((want - base) % 16) + 16) % 16;
            L.lds = L.nseq * L.lstride;
        }
        if (!L.blue && (r.n & (r.n - 1)) == 0) {
            int lg = 0;
            while ((1 << lg) < r.n) ++lg;
            const int S = p2_seqs_per_group(lg);
            if (S > 0) {
                L.p2 = lg;
                L.nseq = S;
                L.lgseq = 0;
                while ((1 << L.lgseq) < S) ++L.lgseq;
                L.ldsc = S * r.n;
                const int base = len + len / 16, want = (16 / L.nseq) % 16;
                L.lstride = base + (((want - base) % 16) + 16) % 16;
                L.lds = L.nseq * L.lstride;
            }
        }
        r.len = (int)p->lens.size();
        len_index[r.n] = r.len;
        if (L.blue) blue.push_back(r.len);
        p->lens.push_back(L);
    }
    Dev drings, dlens, dtw, dbhat, dblue;
    int rc;
    if ((rc = upload(p, drings, p->rings))) return rc;
    if ((rc = upload(p, dlens, p->lens))) return rc;
    if ((rc = upload(p, dtw, pool))) return rc;
    if ((rc = dev_alloc(p, dbhat, std::max<int64_t>(1, bhat_total) * sizeof(double2)))) return rc;
    p->d_rings = (RingDev*)drings.p;
    p->d_lens = (FftLen*)dlens.p;
    p->d_tw = (double2*)dtw.p;
    p->d_bhat = (double2*)dbhat.p;

    if (!blue.empty()) {
        if ((rc = upload(p, dblue, blue))) return rc;
        HIPCHK(launch_bluestein_init(p->d_lens, (const int*)dblue.p, (int)blue.size(), p->d_tw, p->d_bhat,
                                     max_blue_m + max_blue_m / 16 + 1, p->stream));
    }
    return SHT_OK;
}

// FFT work items (ring, first pair) for npairs map pairs, grouped by LDS class.
int build_items(sht_plan p, int npairs)
{
    if (p->items_npairs == npairs) return SHT_OK;
    auto found = p->item_sets.find(npairs);
    if (found != p->item_sets.end()) {
        p->classes = found->second.classes;
        p->items_npairs = npairs;
        return SHT_OK;
    }
    // classes 0..2: runtime-length kernels by LDS size; 3 + (k - 6): length 2^k;
    // 10 + (k - 6): Bluestein through length 2^k; 17: four-step (n = 4j)
    constexpr int NCLS = 3 + 7 + 7 + 1;
    std::vector<FftItem> cls_items[NCLS];
    int lds[NCLS] = {};
    for (int r = 0; r < p->nring; ++r) {
        const FftLen& L = p->lens[p->rings[r].len];
        int c = (L.ldsc <= 2 * FFT_THREADS) ? 0 : (L.ldsc <= 8 * FFT_THREADS ? 1 : 2);
        if (L.p2) c = 3 + (L.p2 - 6);
        if (L.bp2) c = 10 + (L.bp2 - 6);
        if (L.four) c = NCLS - 1;
        lds[c] = std::max(lds[c], L.lds);
        if (npairs % L.nseq) return fail(SHT_ERR_UNSUPPORTED, "map pairs per chunk not a multiple of the ring batch");
        for (int q = 0; q < npairs; q += L.nseq) cls_items[c].push_back(FftItem{r, q});
    }
    std::vector<FftItem> all;
    size_t off[NCLS];
    for (int c = 0; c < NCLS; ++c) { off[c] = all.size(); all.insert(all.end(), cls_items[c].begin(), cls_items[c].end()); }
    sht_plan_s::ItemSet set;
    size_t bytes = std::max<size_t>(1, all.size()) * sizeof(FftItem);
    HIPCHK(hipMalloc(&set.dev.p, bytes));
    set.dev.n = bytes;
    HIPCHK(hipMemcpy(set.dev.p, all.data(), all.size() * sizeof(FftItem), hipMemcpyHostToDevice));
    p->table_bytes += bytes;
    // the residual kernel runs every class with the runtime-length code: the
    // power-of-two classes hold at most 4096 values per workgroup (8 per thread)
    for (int c = 0; c < NCLS; ++c) {
        const int elems = c == 0 ? 2 : (c == 2 ? 16 : 8);
        const int lg = c >= 10 ? c - 10 + 6 : (c >= 3 ? c - 3 + 6 : 0);
        const bool four = (c == NCLS - 1);
        set.classes.push_back(FftClass{(const FftItem*)set.dev.p + off[c], (int)cls_items[c].size(), lds[c], elems,
                                       four ? 0 : lg, (c >= 10 && !four) ? 1 : 0, four ? 1 : 0});
    }
    p->classes = set.classes;
    p->item_sets.emplace(npairs, std::move(set));
    p->items_npairs = npairs;
    return SHT_OK;
}

// --------------------------------------------------------------------------
// Legendre seeds
// --------------------------------------------------------------------------
// scaled form of a value given its log2 magnitude: mu * 2^(-SCALE_BITS k),
// |mu| in [2^SIG_LOG2, 2^(SIG_LOG2 + SCALE_BITS))
void scaled(ld log2abs, double sign, double& mu, int& k)
{
    k = 0;
    if (log2abs < (ld)SIG_LOG2) k = (int)ceill(((ld)SIG_LOG2 - log2abs) / (ld)SCALE_BITS);
    mu = sign * (double)exp2l(log2abs + (ld)SCALE_BITS * k);
}

int build_seeds(sht_plan p, SeedSet& S, int spin)
{
    S.spin = spin;
    const int L = p->lmax, rn = p->rn;
    // start values lambda_{lb}(theta_r) per (m, north ring) in scaled form
    std::vector<double> start((size_t)(spin == 0 ? 1 : 2) * (L + 1) * rn);
    std::vector<int> startk((size_t)(L + 1) * rn);
    if (spin == 0) {
        // lambda_mm = (-1)^m (4 pi)^{-1/2} prod_{k=1}^m sqrt((2k+1)/(2k)) sin^m(theta)
        ld lognorm = -0.5L * log2l(4.0L * PI_L);
        for (int m = 0; m <= L; ++m) {
            if (m > 0) lognorm += 0.5L * log2l((ld)(2 * m + 1) / (ld)(2 * m));
            if (!owns(p, m)) continue;
            double sign = (m & 1) ? -1.0 : 1.0;
            for (int r = 0; r < rn; ++r) {
                ld t = lognorm + (ld)m * log2l((ld)p->rings[r].sth);
                scaled(t, sign, start[(size_t)m * rn + r], startk[(size_t)m * rn + r]);
            }
        }
    } else {
        // {}_{+-2}lambda_{lb} = sqrt((2lb+1)/4pi) d^{lb}_{m,-+2}(theta), lb = max(m, 2)
        for (int m = 0; m <= L; ++m) {
            if (!owns(p, m)) continue;
            int lb = std::max(m, 2);
            ld lnorm = 0.5L * logl((ld)(2 * lb + 1) / (4.0L * PI_L));
            for (int r = 0; r < rn; ++r) {
                // cos^2(theta/2) = (1 + z)/2, sin^2(theta/2) = (1 - z)/2 from the exact 1 - z
                const ld omz = (ld)p->rings[r].omz;
                ld lc = 0.5L * log1pl(-omz / 2.0L), ls = 0.5L * logl(omz / 2.0L);
                ld lP, lM;
                double sP, sM;
                if (m >= 2) {
                    ld f = 0.5L * (lgammal(2.0L * m + 1) - lgammal((ld)m - 1) - lgammal((ld)m + 3));
                    lP = f + (ld)(m - 2) * lc + (ld)(m + 2) * ls;
                    lM = f + (ld)(m + 2) * lc + (ld)(m - 2) * ls;
                    sP = sM = (m & 1) ? -1.0 : 1.0;
                } else {
                    ld f = 0.5L * (logl(24.0L) - lgammal(3.0L - m) - lgammal(3.0L + m));
                    lP = f + (ld)(2 - m) * lc + (ld)(2 + m) * ls;
                    lM = f + (ld)(2 + m) * lc + (ld)(2 - m) * ls;
                    sP = (m & 1) ? -1.0 : 1.0;
                    sM = 1.0;
                }
                lP += lnorm;
                lM += lnorm;
                ld lmax2 = std::max(lP, lM) / logl(2.0L);
                int k = 0;
                if (lmax2 < (ld)SIG_LOG2) k = (int)ceill(((ld)SIG_LOG2 - lmax2) / (ld)SCALE_BITS);
                ld sh = (ld)SCALE_BITS * k * logl(2.0L);
                start[(size_t)m * rn + r] = sP * (double)expl(lP + sh);
                start[(size_t)(L + 1) * rn + (size_t)m * rn + r] = sM * (double)expl(lM + sh);
                startk[(size_t)m * rn + r] = k;
            }
        }
    }
    std::vector<int64_t> seedoff(L + 2), rowoff(L + 2);
    std::vector<int> tileoff(L + 2);
    int64_t tot = 0, rows = 0;
    int tt = 0;
    for (int m = 0; m <= L; ++m) {
        seedoff[m] = tot;
        tileoff[m] = tt;
        rowoff[m] = rows;
        // an m the plan does not own has no seeds, l tiles or coefficient rows
        const int ns = owns(p, m) ? nsegs(spin, L, m) : 0;
        tot += (int64_t)ns * rn;
        tt += (ns + SPT - 1) / SPT;  // l tiles of TL = SPT segments
        rows += owns(p, m) ? std::max(0, L + 1 - lbase(spin, m)) : 0;
    }
    seedoff[L + 1] = tot;
    tileoff[L + 1] = tt;
    rowoff[L + 1] = rows;
    // the same l tiles listed in folded m order (work list of the map2alm kernels)
    std::vector<int> ftileoff(L + 2);
    ftileoff[0] = 0;
    for (int i = 0; i <= L; ++i) {
        const int m = mfold(i, L);
        ftileoff[i + 1] = ftileoff[i] + (tileoff[m + 1] - tileoff[m]);
    }
    S.stride = tot;
    S.ntiles = tt;
    S.rows = rows;
    int rc;
    const int nmu = (spin == 0) ? 2 : 4;
    if ((rc = dev_alloc(p, S.mu, (size_t)std::max<int64_t>(1, tot) * nmu * sizeof(double)))) return rc;
    if ((rc = dev_alloc(p, S.kk, (size_t)std::max<int64_t>(1, tot) * sizeof(int)))) return rc;
    if ((rc = upload(p, S.seedoff, seedoff))) return rc;
    if ((rc = upload(p, S.tileoff, tileoff))) return rc;
    if ((rc = upload(p, S.ftileoff, ftileoff))) return rc;
    if ((rc = upload(p, S.rowoff, rowoff))) return rc;
    const int cstr = (spin == 0) ? 2 : 4;
    const size_t coef_bytes = (size_t)(rows + TL) * cstr * sizeof(double);
    if ((rc = dev_alloc(p, S.coef, coef_bytes))) return rc;
    HIPCHK(hipMemsetAsync(S.coef.p, 0, coef_bytes, p->stream));
    HIPCHK(launch_coefs((double*)S.coef.p, (const int64_t*)S.rowoff.p, L, spin, p->stream));
    if ((rc = dev_alloc(p, S.lsig, (size_t)(L + 1) * p->nrc * sizeof(int)))) return rc;
    HIPCHK(hipMemsetD32Async((hipDeviceptr_t)S.lsig.p, L + 1, (size_t)(L + 1) * p->nrc, p->stream));
    void* d_start = nullptr;
    void* d_startk = nullptr;
    HIPCHK(hipMalloc(&d_start, start.size() * sizeof(double)));
    HIPCHK(hipMalloc(&d_startk, startk.size() * sizeof(int)));
    HIPCHK(hipMemcpy(d_start, start.data(), start.size() * sizeof(double), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(d_startk, startk.data(), startk.size() * sizeof(int), hipMemcpyHostToDevice));
    SeedArgs a{};
    a.rings = p->d_rings;
    a.start = (const double*)d_start;
    a.startk = (const int*)d_startk;
    a.mu = (double*)S.mu.p;
    a.kk = (int*)S.kk.p;
    a.seedoff = (const int64_t*)S.seedoff.p;
    a.seedstride = S.stride;
    a.lsig = (int*)S.lsig.p;
    a.nrc = p->nrc;
    a.lmax = L;
    a.rn = rn;
    a.spin = spin;
    hipError_t e = launch_seeds(a, p->stream);
    hipError_t e2 = hipStreamSynchronize(p->stream);
    (void)hipFree(d_start);
    (void)hipFree(d_startk);
    HIPCHK(e);
    HIPCHK(e2);
    return SHT_OK;
}

// Ring optimisation in the FFT mapping (Sec. 3.1 item 10): the Legendre kernels
// skip ring chunks whose values are all negligible for an m, and map2alm reads a
// ring chunk c for m only from the first significant chunk of that m on, so rows
// (m, ring) past mcut(c) = max{m : first significant chunk of m <= c} are never
// read, and alm2map leaves them exactly zero (negligible values are emitted as
// zeros).  The ring FFTs therefore unfold and fold only m <= mcut of the ring's
// chunk, the larger of the two spins' bounds.
int build_mcut(sht_plan p)
{
    const int L = p->lmax, nrc = p->nrc;
    std::vector<int> mcut(nrc, 0), lsig((size_t)(L + 1) * nrc);
    p->cmin.assign(L + 1, nrc);
    for (SeedSet* S : {&p->s0, &p->s2}) {
        if (!S->lsig.p) continue;
        HIPCHK(hipMemcpy(lsig.data(), S->lsig.p, lsig.size() * sizeof(int), hipMemcpyDeviceToHost));
        for (int m = 0; m <= L; ++m) {
            int c = 0;
            while (c < nrc && lsig[(size_t)m * nrc + c] > L) ++c;
            for (int cc = c; cc < nrc; ++cc) mcut[cc] = std::max(mcut[cc], m);
            p->cmin[m] = std::min(p->cmin[m], c);
        }
    }
    for (int r = 0; r < p->nring; ++r) {
        const int rn = std::min(r, p->nring - 1 - r);
        p->rings[r].mcut = mcut[rn / RCHUNK];
    }
    HIPCHK(hipMemcpy(p->d_rings, p->rings.data(), p->rings.size() * sizeof(RingDev), hipMemcpyHostToDevice));
    return SHT_OK;
}

// --------------------------------------------------------------------------
// workspace
// --------------------------------------------------------------------------
// element size of the ring coefficients X and of the rows map2alm writes
size_t esize(int prec) { return prec == SHT_FP64 ? sizeof(double) : sizeof(float); }
// bytes per element of a separate alm2map operand region: split-BF16 words (the
// other precisions read the map2alm rows' own region)
size_t opsize(int prec) { return prec == SHT_BF16X3 ? sizeof(uint64_t) : 0; }

// columns of the m-major operand arrays: 2 * map sets, padded to 32 map sets for
// batches of up to 32 (one 64-column tile) and to a multiple of 64 beyond
int64_t ldx_for(int chunk) { return chunk <= 32 ? 64 : 2 * (int64_t)((chunk + 63) / 64 * 64); }

int64_t xcomp_elems(sht_plan p) { return (int64_t)(p->lmax + 1) * p->nring * ldx_for(p->chunk); }

// rows of the m-major coefficient arrays (spin-0 count bounds the spin-2 one)
int64_t acomp_elems(sht_plan p)
{
    int64_t L = p->lmax;
    return (L + 1) * (L + 2) / 2 * ldx_for(p->chunk);
}

// workspace bytes for chunks of `chunk` map sets in precision `prec`
size_t ws_need_at(sht_plan p, int chunk, int prec)
{
    const int64_t L = p->lmax, ldx = ldx_for(chunk);
    const size_t x = (size_t)(L + 1) * p->nring * ldx, a = (size_t)((L + 1) * (L + 2) / 2) * ldx;
    return (size_t)p->ncomp * ((x + a) * esize(prec) + a * opsize(prec));
}

size_t ws_need(sht_plan p) { return ws_need_at(p, p->chunk, p->prec); }

// largest chunk (at most the plan's capacity) whose workspace fits the static
// workspace in precision `prec`; 0 if one map set does not fit
int noalloc_chunk(sht_plan p, int prec)
{
    int lo = 0, hi = p->cap;
    while (lo < hi) {  // ws_need_at grows with the chunk
        const int mid = lo + (hi - lo + 1) / 2;
        if (ws_need_at(p, mid, prec) <= SCRATCH_BYTES) lo = mid; else hi = mid - 1;
    }
    return lo;
}

void* ws_A(sht_plan p) { return (char*)p->ws + (size_t)p->ncomp * xcomp_elems(p) * esize(p->prec); }
// the alm2map operand rows: the map2alm rows' region, or the split-BF16 words after it
void* ws_Aop(sht_plan p)
{
    if (!opsize(p->prec)) return ws_A(p);
    return (char*)ws_A(p) + (size_t)p->ncomp * acomp_elems(p) * esize(p->prec);
}

int default_chunk(sht_plan p)
{
    const double budget = 8.0e9;
    double per = (double)p->ncomp * (p->lmax + 1) * 2.0 *
                 ((p->nring + (p->lmax + 2) / 2.0) * esize(p->prec) + (p->lmax + 2) / 2.0 * opsize(p->prec));
    int c = (int)std::max(1.0, std::floor(budget / per));
    if (c >= 64) c = c / 64 * 64;
    return std::min(c, p->cap);
}

int ensure_workspace(sht_plan p)
{
    size_t need = ws_need(p);
    if (p->ws && p->ws_bytes >= need) return SHT_OK;
    if (p->ws && !p->ws_owned)
        return fail(SHT_ERR_ARG, "caller workspace of " + std::to_string(p->ws_bytes) + " bytes is smaller than the " +
                                     std::to_string(need) + " bytes needed");
    if (p->ws) { (void)hipFree(p->ws); p->ws = nullptr; p->ws_bytes = 0; }
    hipError_t e = hipMalloc(&p->ws, need);
    if (e != hipSuccess) {
        p->ws = nullptr;
        return fail(SHT_ERR_NOMEM, "workspace hipMalloc of " + std::to_string(need) + " bytes failed");
    }
    p->ws_bytes = need;
    p->ws_owned = true;
    return SHT_OK;
}

int ensure_iter_buffers(sht_plan p)
{
    size_t need = (size_t)p->chunk * p->ncomp * (size_t)p->npix * sizeof(double);
    if (p->F && p->F_bytes >= need) return SHT_OK;
    if (p->F) (void)hipFree(p->F);
    if (p->norms) (void)hipFree(p->norms);
    p->F = nullptr;
    p->norms = nullptr;
    HIPCHK(hipMalloc((void**)&p->F, need));
    HIPCHK(hipMalloc((void**)&p->norms, (size_t)p->chunk * p->ncomp * sizeof(double) + 64));
    p->F_bytes = need;
    return SHT_OK;
}

// --------------------------------------------------------------------------
// kernel argument assembly
// --------------------------------------------------------------------------
FftArgs fft_args(sht_plan p, int nmaps_chunk)
{
    FftArgs a{};
    a.rings = p->d_rings;
    a.lens = p->d_lens;
    a.tw = p->d_tw;
    a.bhat = p->d_bhat;
    a.X = p->ws;
    a.npix = p->npix;
    a.ncomp = p->ncomp;
    a.comp0 = 0;
    a.nmaps = nmaps_chunk;
    a.ldx = p->ldx_cur;
    a.npairs = (int)(a.ldx / 4);
    a.lmax = p->lmax;
    a.nring = p->nring;
    a.xcomp = xcomp_elems(p);
    a.x32 = (p->prec != SHT_FP64);
    a.mown = p->nparts > 1 ? (const unsigned char*)p->d_own.p : nullptr;
    return a;
}

LegArgs leg_args(sht_plan p, const SeedSet& S)
{
    LegArgs a{};
    a.ncols = 2 * p->nm_cur;
    a.rings = p->d_rings;
    a.mu = (const double*)S.mu.p;
    a.kk = (const int*)S.kk.p;
    a.seedoff = (const int64_t*)S.seedoff.p;
    a.seedstride = S.stride;
    a.lsig = (const int*)S.lsig.p;
    a.nrc = p->nrc;
    a.tiles = (const int*)S.ftileoff.p;
    a.ntiles = S.ntiles;
    a.X = p->ws;
    a.xcomp = xcomp_elems(p);
    a.A = ws_A(p);
    a.acomp = acomp_elems(p);
    a.rowoff = (const int64_t*)S.rowoff.p;
    a.coef = (const double*)S.coef.p;
    a.ldx = p->ldx_cur;
    a.lmax = p->lmax;
    a.rn = p->rn;
    a.nring = p->nring;
    a.spin = S.spin;
    return a;
}

AlmArgs alm_args(sht_plan p, const SeedSet& S, int nmaps_chunk)
{
    AlmArgs a{};
    a.A = ws_A(p);
    a.Aop = ws_Aop(p);
    a.acomp = acomp_elems(p);
    a.rowoff = (const int64_t*)S.rowoff.p;
    a.tileoff = (const int*)S.tileoff.p;
    a.ntiles = S.ntiles;
    a.ldx = p->ldx_cur;
    a.kblocks = (int)(a.ldx / 64);
    a.almstride = (int64_t)p->ncomp * (p->lmax + 1) * (p->lmax + 1);
    a.lmax = p->lmax;
    a.spin = S.spin;
    a.nmaps = nmaps_chunk;
    a.comp0 = (S.spin == 0) ? 0 : 1;
    a.scale = 1.0;
    return a;
}

int prep(sht_plan p)
{
    int rc = ensure_workspace(p);
    if (rc) return rc;
    p->ldx_cur = ldx_for(p->chunk);
    p->nm_cur = p->chunk;
    return build_items(p, (int)(p->ldx_cur / 4));
}

// Narrow the m-major row pitch to what a chunk of nm map sets needs (a last,
// partial chunk then computes only its own columns); the component arrays keep
// the full chunk's spacing, so any narrower pitch fits the workspace.
int use_width(sht_plan p, int nm)
{
    p->ldx_cur = ldx_for(nm);
    p->nm_cur = nm;
    return build_items(p, (int)(p->ldx_cur / 4));
}

// Component selection (enum sht_comp bits) of the selective transforms.  The
// spin-2 block row kept by E-only / B-only (Sec. 2.3: the 0/1 diagonal selector
// lambda^{E,B}) goes to the Legendre kernels as LegArgs::eb.
bool sel_t(int sel) { return (sel & SHT_COMP_T) != 0; }
bool sel_pol(sht_plan p, int sel) { return p->spin == 2 && (sel & (SHT_COMP_E | SHT_COMP_B)) != 0; }
int sel_eb(int sel)
{
    const int eb = sel & (SHT_COMP_E | SHT_COMP_B);
    return eb == SHT_COMP_E ? 1 : eb == SHT_COMP_B ? 2 : 0;
}

int valid_sel(sht_plan p, int sel)
{
    if (sel == 0 || (sel & ~SHT_COMP_ALL)) return fail(SHT_ERR_ARG, "component selection must be a nonzero mask of SHT_COMP_T/E/B");
    if (p->spin == 0 && sel != SHT_COMP_T) return fail(SHT_ERR_ARG, "a spin-0 plan has only the T component");
    return SHT_OK;
}

// compact alm -> m-major operand rows for the selected components
int run_to_mmajor(sht_plan p, const double* alm, int nm, int sel)
{
    StageTimer t(p, SHT_STAGE_ALM_LAYOUT);
    if (sel_t(sel)) {
        AlmArgs t0 = alm_args(p, p->s0, nm);
        t0.alm_in = alm;
        HIPCHK(launch_alm_to_mmajor(t0, 1, p->prec, p->stream));
    }
    if (sel_pol(p, sel)) {
        AlmArgs t2 = alm_args(p, p->s2, nm);
        t2.alm_in = alm;
        const int eb = sel_eb(sel);
        if (eb == 2) t2.comp0 = 2;
        HIPCHK(launch_alm_to_mmajor(t2, eb ? 1 : 2, p->prec, p->stream));
    }
    return SHT_OK;
}

// a plan owning part of the m runs the alm2map kernels on its m list (the
// map2alm kernels and the layout kernels find no tiles for the other m)
void own_list(sht_plan p, LegArgs& a)
{
    if (p->nparts <= 1) return;
    a.mlist = (const int*)p->d_mlist.p;
    a.nlist = p->nown;
}

// m-major rows -> ring Fourier coefficients of the selected components
int run_leg_a2m(sht_plan p, int sel)
{
    if (sel_t(sel)) {
        StageTimer t(p, SHT_STAGE_A2M_SPIN0);
        LegArgs a = leg_args(p, p->s0);
        a.A = ws_Aop(p);
        own_list(p, a);
        HIPCHK(launch_leg_a2m(a, p->prec, p->stream));
    }
    if (sel_pol(p, sel)) {
        StageTimer t(p, SHT_STAGE_A2M_SPIN2);
        LegArgs a = leg_args(p, p->s2);
        a.A = ws_Aop(p);
        own_list(p, a);
        a.eb = sel_eb(sel);
        HIPCHK(launch_leg_a2m(a, p->prec, p->stream));
    }
    return SHT_OK;
}

int run_a2m(sht_plan p, const double* alm, int nm, int sel = SHT_COMP_ALL)
{
    int rc = run_to_mmajor(p, alm, nm, sel);
    return rc ? rc : run_leg_a2m(p, sel);
}

// Inverse ring FFTs of the selected components into maps; components left out
// are written as zero.
int run_fft_inv(sht_plan p, double* maps, int nm, int sel)
{
    FftArgs f = fft_args(p, nm);
    f.maps_out = maps;
    const bool t = sel_t(sel), pol = sel_pol(p, sel);
    const int64_t mstride = (int64_t)p->ncomp * p->npix;
    int ncompl = p->ncomp;
    if (p->spin == 2 && !(t && pol)) {
        f.comp0 = t ? 0 : 1;
        ncompl = t ? 1 : 2;
        double* zb = t ? maps + p->npix : maps;
        HIPCHK(launch_zero_strided(zb, nm, mstride, (int64_t)(3 - ncompl) * p->npix, p->stream));
    }
    StageTimer tm(p, SHT_STAGE_FFT_INV);
    HIPCHK(launch_fft_inverse(f, p->classes.data(), (int)p->classes.size(), ncompl, p->stream));
    return SHT_OK;
}

int run_m2a(sht_plan p, double* alm, int nm, int accumulate, int sel = SHT_COMP_ALL)
{
    const double dsig = 4.0 * M_PI / (double)p->npix;
    const bool t = sel_t(sel), pol = sel_pol(p, sel);
    if (t) {
        StageTimer tm(p, SHT_STAGE_M2A_SPIN0);
        HIPCHK(launch_leg_m2a(leg_args(p, p->s0), p->prec, p->stream));
    }
    if (pol) {
        StageTimer tm(p, SHT_STAGE_M2A_SPIN2);
        LegArgs a = leg_args(p, p->s2);
        a.eb = sel_eb(sel);
        HIPCHK(launch_leg_m2a(a, p->prec, p->stream));
    }
    StageTimer tm(p, SHT_STAGE_ALM_LAYOUT);
    const int64_t csz = (int64_t)(p->lmax + 1) * (p->lmax + 1);
    const int64_t astride = (int64_t)p->ncomp * csz;
    if (t) {
        AlmArgs t0 = alm_args(p, p->s0, nm);
        t0.alm_out = alm;
        t0.scale = dsig;
        t0.accumulate = accumulate;
        HIPCHK(launch_alm_from_mmajor(t0, 1, p->prec, p->stream));
    } else if (!accumulate) {
        HIPCHK(launch_zero_strided(alm, nm, astride, csz, p->stream));
    }
    if (pol) {
        // with E or B alone the kernel leaves the other block's rows zero
        AlmArgs t2 = alm_args(p, p->s2, nm);
        t2.alm_out = alm;
        t2.scale = dsig;
        t2.accumulate = accumulate;
        HIPCHK(launch_alm_from_mmajor(t2, 2, p->prec, p->stream));
    } else if (p->spin == 2 && !accumulate) {
        HIPCHK(launch_zero_strided(alm + csz, nm, astride, 2 * csz, p->stream));
    }
    return SHT_OK;
}

// Schedule of the immediate iteration (Sec. 4, Algorithm 3): a Gauss-Seidel
// sweep over m in increasing order.  The update of m changes the residual only in
// bins m mod n and -m mod n of the rings where m carries data, and the analysis
// of m reads only those bins, so m depends on exactly the earlier m that share
// such a bin on such a ring.  Level(m) = 1 + the highest level among them: the m
// of one level are independent and run together, and running the levels in
// order gives the sweep's result (up to the order of floating-point additions).
int build_levels(sht_plan p)
{
    auto& V = p->lev;
    if (V.built) return SHT_OK;
    const int L = p->lmax, rn = p->rn;
    std::vector<int64_t> off(rn + 1, 0);  // per north ring: slots for bins 0 .. n/2
    for (int r = 0; r < rn; ++r) off[r + 1] = off[r] + p->rings[r].n / 2 + 1;
    std::vector<int> last(off[rn], 0), level(L + 1, 0);
    int depth = 0;
    for (int m = 0; m <= L; ++m) {
        const int r0 = std::min(rn, p->cmin[m] * RCHUNK);
        int lv = 0;
        for (int r = r0; r < rn; ++r) {
            const int n = p->rings[r].n, j = m % n;
            lv = std::max(lv, last[off[r] + std::min(j, n - j)]);
        }
        level[m] = ++lv;
        depth = std::max(depth, lv);
        for (int r = r0; r < rn; ++r) {
            const int n = p->rings[r].n, j = m % n;
            last[off[r] + std::min(j, n - j)] = lv;
        }
    }
    std::vector<std::vector<int>> by(depth);
    for (int m = 0; m <= L; ++m) by[level[m] - 1].push_back(m);
    std::vector<int> mlist, pref0, pref2;
    auto ntl = [&](int spin, int m) { const int lb = lbase(spin, m); return lb > L ? 0 : (L - lb + TL) / TL; };
    for (int d = 0; d < depth; ++d) {
        V.start.push_back((int)mlist.size());
        V.len.push_back((int)by[d].size());
        int t0 = 0, t2 = 0;
        pref0.push_back(0);
        pref2.push_back(0);
        for (int m : by[d]) {
            mlist.push_back(m);
            pref0.push_back(t0 += ntl(0, m));
            pref2.push_back(t2 += ntl(2, m));
        }
        V.ntiles0.push_back(t0);
        V.ntiles2.push_back(t2);
    }
    int rc;
    if ((rc = upload(p, V.mlist, mlist))) return rc;
    if ((rc = upload(p, V.pref0, pref0))) return rc;
    if ((rc = upload(p, V.pref2, pref2))) return rc;
    if ((rc = upload(p, V.cmin, p->cmin))) return rc;
    V.built = true;
    return SHT_OK;
}

// One level of an immediate sweep on the chunk's residual spectra (in p->R):
// unfold R for the listed m, analyse, add dsigma times the result to alm, turn
// the rows into the synthesis operand of the update, synthesise, fold back.
int run_level(sht_plan p, double* alm, int nm, int d)
{
    auto& V = p->lev;
    const int* ml = (const int*)V.mlist.p + V.start[d];
    const int nl = V.len[d];
    const double dsig = 4.0 * M_PI / (double)p->npix;
    FftArgs f = fft_args(p, nm);
    f.R = p->R;
    {
        StageTimer t(p, SHT_STAGE_RESIDUAL);
        HIPCHK(launch_level_unfold(f, ml, nl, (const int*)V.cmin.p, p->ncomp, p->stream));
    }
    // A level holds a few m, so its Legendre grids would cover a fraction of the
    // chip with long serial reductions: split each reduction over several
    // workgroups (about 1024 per launch) that add into cleared outputs.
    const int ct = (int)std::max<int64_t>(1, p->ldx_cur / 128);
    auto parts = [](int64_t wgs) { return (int)std::min<int64_t>(8, std::max<int64_t>(1, 1024 / std::max<int64_t>(1, wgs))); };
    for (int spin : {0, 2}) {
        if (spin == 2 && p->spin != 2) break;
        SeedSet& S = spin == 0 ? p->s0 : p->s2;
        const int* pref = (const int*)(spin == 0 ? V.pref0.p : V.pref2.p) + V.start[d] + d;
        const int nt = spin == 0 ? V.ntiles0[d] : V.ntiles2[d];
        const int ncompl = spin == 0 ? 1 : 2;
        LegArgs a = leg_args(p, S);
        a.mlist = ml;
        a.nlist = nl;
        a.tiles = pref;
        a.ntiles = nt;
        AlmArgs b = alm_args(p, S, nm);
        b.mlist = ml;
        b.nlist = nl;
        b.tileoff = pref;
        b.ntiles = nt;
        b.alm_out = alm;
        b.accumulate = 1;
        {
            StageTimer t(p, spin == 0 ? SHT_STAGE_M2A_SPIN0 : SHT_STAGE_M2A_SPIN2);
            a.ksplit = parts((int64_t)nt * ct);
            if (a.ksplit > 1) {
                b.scale = 0.0;  // clear the rows the split map2alm adds into
                HIPCHK(launch_level_rows(b, ncompl, p->prec, p->stream));
            }
            HIPCHK(launch_leg_m2a(a, p->prec, p->stream));
        }
        {
            StageTimer t(p, SHT_STAGE_ALM_LAYOUT);
            b.scale = dsig;
            HIPCHK(launch_level_commit(b, ncompl, p->prec, p->stream));
        }
        {
            StageTimer t(p, spin == 0 ? SHT_STAGE_A2M_SPIN0 : SHT_STAGE_A2M_SPIN2);
            const int tr = spin == 0 ? 64 : 32;  // rings per alm2map tile
            a.ksplit = parts((int64_t)nl * ct * ((p->rn + tr - 1) / tr));
            if (a.ksplit > 1) {  // clear this spin's rows the split alm2map adds into
                FftArgs z = f;
                z.comp0 = spin == 0 ? 0 : 1;
                HIPCHK(launch_level_zero(z, ml, nl, ncompl, p->stream));
            }
            a.A = ws_Aop(p);  // the rows the commit wrote as the synthesis operand
            HIPCHK(launch_leg_a2m(a, p->prec, p->stream));
        }
    }
    StageTimer t(p, SHT_STAGE_RESIDUAL);
    HIPCHK(launch_level_fold(f, ml, nl, (const int*)V.cmin.p, p->ncomp, p->stream));
    return SHT_OK;
}

// the calls a plan owning part of the m does not offer
int whole_only(sht_plan p, const char* what)
{
    if (p && p->nparts > 1)
        return fail(SHT_ERR_UNSUPPORTED, std::string(what) + " needs a plan of all orders m (sht_plan_create)");
    return SHT_OK;
}

int check_ready(sht_plan p)
{
    if (!p) return fail(SHT_ERR_ARG, "null plan");
    int dev = -1;
    HIPCHK(hipGetDevice(&dev));
    if (dev != p->device) return fail(SHT_ERR_ARG, "current HIP device differs from the plan's device");
    HIPCHK(hipGetLastError());
    return SHT_OK;
}

void drop_records(sht_plan p)
{
    for (auto& r : p->recs) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    p->recs.clear();
}

void destroy_all(sht_plan p)
{
    drop_records(p);
    for (auto& d : p->owned)
        if (d.p) (void)hipFree(d.p);
    for (auto& kv : p->item_sets)
        if (kv.second.dev.p) (void)hipFree(kv.second.dev.p);
    if (p->ws && p->ws_owned) (void)hipFree(p->ws);
    if (p->F) (void)hipFree(p->F);
    if (p->norms) (void)hipFree(p->norms);
    if (p->R) (void)hipFree(p->R);
    delete p;
}

}  // namespace

// ============================================================================
// C ABI
// ============================================================================
extern "C" {

const char* sht_last_error(void) { return g_err.c_str(); }

}  // extern "C"

namespace {

int create_plan(sht_plan* out, int nside, int lmax, int spin, int nmaps, int part, int nparts)
{
    g_err.clear();
    if (!out) return fail(SHT_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (nside < 1 || nside > 8192) return fail(SHT_ERR_ARG, "nside must be in [1, 8192]");
    if (lmax < 0 || lmax > 4 * nside - 1) return fail(SHT_ERR_ARG, "lmax must be in [0, 4*nside-1]");
    if (spin != 0 && spin != 2) return fail(SHT_ERR_ARG, "spin must be 0 or 2");
    if (spin == 2 && lmax < 2) return fail(SHT_ERR_ARG, "spin 2 needs lmax >= 2");
    if (nmaps < 1) return fail(SHT_ERR_ARG, "nmaps must be >= 1");
    if (nparts < 1 || part < 0 || part >= nparts) return fail(SHT_ERR_ARG, "part must be in [0, nparts)");
    if (nside > 2048) return fail(SHT_ERR_UNSUPPORTED, "nside above 2048 is not supported (ring FFT LDS plan)");
    sht_plan p = new sht_plan_s();
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) { delete p; return fail(SHT_ERR_DEVICE, "no HIP device"); }
    p->device = dev;
    p->nside = nside;
    p->lmax = lmax;
    p->spin = spin;
    p->ncomp = (spin == 0) ? 1 : 3;
    p->cap = nmaps;
    p->nmaps = nmaps;
    p->stream = nullptr;
    p->part = part;
    p->nparts = nparts;
    std::vector<int> mlist;
    if (nparts > 1) {
        p->own.assign(lmax + 1, 0);
        for (int i = 0; i <= lmax; ++i)
            if ((i >> 1) % nparts == part) p->own[mfold(i, lmax)] = 1;
        for (int m = 0; m <= lmax; ++m)
            if (p->own[m]) mlist.push_back(m);
        p->nown = (int)mlist.size();
    } else {
        p->nown = lmax + 1;
    }
    build_rings(p);
    p->nrc = (p->rn + RCHUNK - 1) / RCHUNK;
    int rc = build_fft(p);
    if (!rc && nparts > 1) rc = upload(p, p->d_own, p->own);
    if (!rc && nparts > 1) rc = upload(p, p->d_mlist, mlist);
    if (!rc && p->nown == 0) rc = fail(SHT_ERR_ARG, "this part owns no order m (more parts than m pairs)");
    if (!rc) rc = build_seeds(p, p->s0, 0);
    if (!rc && spin == 2) rc = build_seeds(p, p->s2, 2);
    if (!rc) rc = build_mcut(p);
    if (!rc) {
        p->chunk = default_chunk(p);
        rc = prep(p);
    }
    // the static workspace of sht_alm2map_noalloc and the FFT work lists of every
    // chunk width it may use, so that call allocates nothing
    if (!rc) rc = resolve_scratch(dev, &p->scratch);
    if (!rc) {
        std::vector<int64_t> widths;
        for (int k = 1; k <= noalloc_chunk(p, SHT_FP32); ++k)
            if (widths.empty() || widths.back() != ldx_for(k)) widths.push_back(ldx_for(k));
        for (size_t i = 0; i < widths.size() && !rc; ++i) rc = build_items(p, (int)(widths[i] / 4));
        if (!rc) rc = build_items(p, (int)(p->ldx_cur / 4));
    }
    if (!rc) {
        hipError_t e = hipStreamSynchronize(p->stream);
        if (e != hipSuccess) rc = fail(SHT_ERR_DEVICE, std::string("plan set-up: ") + hipGetErrorString(e));
    }
    if (rc) { destroy_all(p); return rc; }
    *out = p;
    return SHT_OK;
}

}  // namespace

extern "C" {

int sht_plan_create(sht_plan* out, int nside, int lmax, int spin, int nmaps)
{
    return create_plan(out, nside, lmax, spin, nmaps, 0, 1);
}

int sht_plan_create_part(sht_plan* out, int nside, int lmax, int spin, int nmaps, int part, int nparts)
{
    return create_plan(out, nside, lmax, spin, nmaps, part, nparts);
}

int sht_plan_destroy(sht_plan p)
{
    if (!p) return SHT_OK;
    (void)hipStreamSynchronize(p->stream);
    destroy_all(p);
    return SHT_OK;
}

int sht_plan_set_precision(sht_plan p, int prec)
{
    if (!p) return fail(SHT_ERR_ARG, "null plan");
    if (prec != SHT_FP64 && prec != SHT_FP32 && prec != SHT_BF16X3) return fail(SHT_ERR_ARG, "unknown precision");
    const int old = p->prec;
    p->prec = prec;
    const int rc = prep(p);
    if (rc != SHT_OK) {  // as in sht_plan_set_chunk: keep what the workspace was sized for
        p->prec = old;
        (void)prep(p);
    }
    return rc;
}

int sht_plan_set_stream(sht_plan p, void* s)
{
    if (!p) return fail(SHT_ERR_ARG, "null plan");
    p->stream = (hipStream_t)s;
    return SHT_OK;
}

int sht_plan_set_nmaps(sht_plan p, int n)
{
    if (!p) return fail(SHT_ERR_ARG, "null plan");
    if (n < 1 || n > p->cap) return fail(SHT_ERR_ARG, "nmaps must be in [1, capacity]");
    p->nmaps = n;
    return SHT_OK;
}

int sht_plan_set_chunk(sht_plan p, int c)
{
    if (!p) return fail(SHT_ERR_ARG, "null plan");
    if (c < 1) return fail(SHT_ERR_ARG, "chunk must be >= 1");
    const int old = p->chunk;
    p->chunk = std::min(c, p->cap);
    const int rc = prep(p);
    if (rc != SHT_OK) {
        // keep the chunk the workspace was sized for (a caller workspace too small
        // for the new one, or a failed allocation); the error of the request stays
        p->chunk = old;
        (void)prep(p);
    }
    return rc;
}

size_t sht_plan_workspace_bytes(sht_plan p) { return p ? ws_need(p) : 0; }

size_t sht_plan_table_bytes(sht_plan p) { return p ? p->table_bytes : 0; }

long long sht_plan_ring_rows(sht_plan p)
{
    if (!p) return 0;
    long long rows = 0;
    for (const RingDev& r : p->rings) rows += std::min(p->lmax, r.mcut) + 1;
    return rows;
}

int sht_plan_set_workspace(sht_plan p, void* ptr, size_t bytes)
{
    if (!p) return fail(SHT_ERR_ARG, "null plan");
    if (ptr && ((uintptr_t)ptr & 255) != 0) return fail(SHT_ERR_ARG, "workspace must be 256-byte aligned");
    if (ptr && bytes < ws_need(p)) return fail(SHT_ERR_ARG, "workspace too small");
    if (p->ws && p->ws_owned) (void)hipFree(p->ws);
    p->ws = ptr;
    p->ws_bytes = ptr ? bytes : 0;
    p->ws_owned = false;
    if (!ptr) return ensure_workspace(p);
    return SHT_OK;
}

int sht_alm2map_sel(sht_plan p, int comps, const double* alm, double* map)
{
    int rc = check_ready(p);
    if (rc) return rc;
    if (!alm || !map) return fail(SHT_ERR_ARG, "null data pointer");
    if ((rc = valid_sel(p, comps))) return rc;
    if (comps != (p->spin == 0 ? SHT_COMP_T : SHT_COMP_ALL) && (rc = whole_only(p, "a component selection")))
        return rc;
    if ((rc = prep(p))) return rc;
    const int64_t astride = (int64_t)p->ncomp * (p->lmax + 1) * (p->lmax + 1);
    const int64_t mstride = (int64_t)p->ncomp * p->npix;
    for (int k0 = 0; k0 < p->nmaps; k0 += p->chunk) {
        int nm = std::min(p->chunk, p->nmaps - k0);
        if ((rc = use_width(p, nm))) return rc;
        if ((rc = run_a2m(p, alm + k0 * astride, nm, comps))) return rc;
        if ((rc = run_fft_inv(p, map + k0 * mstride, nm, comps))) return rc;
    }
    return SHT_OK;
}

int sht_alm2map_noalloc(sht_plan p, const double* alm, double* map)
{
    int rc = check_ready(p);
    if (rc) return rc;
    if ((rc = whole_only(p, "the allocation-free synthesis"))) return rc;
    if (!alm || !map) return fail(SHT_ERR_ARG, "null data pointer");
    if (!p->scratch) return fail(SHT_ERR_DEVICE, "static workspace not resolved on this device");
    const int c = noalloc_chunk(p, p->prec);
    if (c < 1)
        return fail(SHT_ERR_ARG, "the workspace of one map set (" + std::to_string(ws_need_at(p, 1, p->prec)) +
                                     " bytes) exceeds the static workspace of " + std::to_string(SCRATCH_BYTES) +
                                     " bytes");
    for (int k0 = 0; k0 < p->nmaps; k0 += c) {  // every width's work list exists (plan creation)
        const int npairs = (int)(ldx_for(std::min(c, p->nmaps - k0)) / 4);
        if (!p->item_sets.count(npairs)) return fail(SHT_ERR_UNSUPPORTED, "no FFT work list for this chunk width");
    }
    // run the plan's own stages on the static workspace, with chunks of c map sets,
    // no stage timing (events), then give the plan back its own workspace
    void* const ws = p->ws;
    const size_t ws_bytes = p->ws_bytes;
    const bool ws_owned = p->ws_owned, profiling = p->profiling;
    const int chunk = p->chunk, nm_cur = p->nm_cur;
    const int64_t ldx = p->ldx_cur;
    p->ws = p->scratch;
    p->ws_bytes = SCRATCH_BYTES;
    p->ws_owned = false;
    p->profiling = false;
    p->chunk = c;
    const int64_t astride = (int64_t)p->ncomp * (p->lmax + 1) * (p->lmax + 1);
    const int64_t mstride = (int64_t)p->ncomp * p->npix;
    for (int k0 = 0; k0 < p->nmaps && !rc; k0 += c) {
        const int nm = std::min(c, p->nmaps - k0);
        rc = use_width(p, nm);
        if (!rc) rc = run_a2m(p, alm + k0 * astride, nm, SHT_COMP_ALL);
        if (!rc) rc = run_fft_inv(p, map + k0 * mstride, nm, SHT_COMP_ALL);
    }
    p->ws = ws;
    p->ws_bytes = ws_bytes;
    p->ws_owned = ws_owned;
    p->profiling = profiling;
    p->chunk = chunk;
    p->ldx_cur = ldx;
    p->nm_cur = nm_cur;
    const int rc2 = build_items(p, (int)(ldx / 4));  // cached: selects the plan's list again
    return rc ? rc : rc2;
}

int sht_alm2map(sht_plan p, const double* alm, double* map)
{
    return sht_alm2map_sel(p, p && p->spin == 0 ? SHT_COMP_T : SHT_COMP_ALL, alm, map);
}

int sht_map2alm_sel(sht_plan p, int comps, const double* map, double* alm)
{
    int rc = check_ready(p);
    if (rc) return rc;
    if (!alm || !map) return fail(SHT_ERR_ARG, "null data pointer");
    if ((rc = valid_sel(p, comps))) return rc;
    if (comps != (p->spin == 0 ? SHT_COMP_T : SHT_COMP_ALL) && (rc = whole_only(p, "a component selection")))
        return rc;
    if ((rc = prep(p))) return rc;
    const int64_t astride = (int64_t)p->ncomp * (p->lmax + 1) * (p->lmax + 1);
    const int64_t mstride = (int64_t)p->ncomp * p->npix;
    for (int k0 = 0; k0 < p->nmaps; k0 += p->chunk) {
        int nm = std::min(p->chunk, p->nmaps - k0);
        if ((rc = use_width(p, nm))) return rc;
        FftArgs f = fft_args(p, nm);
        f.maps_in = map + k0 * mstride;
        int ncompl = p->ncomp;
        if (p->spin == 2 && !(sel_t(comps) && sel_pol(p, comps))) {
            f.comp0 = sel_t(comps) ? 0 : 1;
            ncompl = sel_t(comps) ? 1 : 2;
        }
        {
            StageTimer t(p, SHT_STAGE_FFT_FWD);
            HIPCHK(launch_fft_forward(f, p->classes.data(), (int)p->classes.size(), ncompl, p->stream));
        }
        if ((rc = run_m2a(p, alm + k0 * astride, nm, 0, comps))) return rc;
    }
    return SHT_OK;
}

int sht_map2alm(sht_plan p, const double* map, double* alm)
{
    return sht_map2alm_sel(p, p && p->spin == 0 ? SHT_COMP_T : SHT_COMP_ALL, map, alm);
}

int sht_eb_split(sht_plan p, const double* map, double* alm, double* map_e, double* map_b)
{
    int rc = check_ready(p);
    if (rc) return rc;
    if ((rc = whole_only(p, "E/B separation"))) return rc;
    if (!map || !alm || !map_e || !map_b) return fail(SHT_ERR_ARG, "null data pointer");
    if (p->spin != 2) return fail(SHT_ERR_ARG, "E/B separation needs a spin-2 plan");
    if (map_e == map_b) return fail(SHT_ERR_ARG, "map_e and map_b must be distinct arrays");
    if ((rc = prep(p))) return rc;
    const int64_t astride = (int64_t)p->ncomp * (p->lmax + 1) * (p->lmax + 1);
    const int64_t mstride = (int64_t)p->ncomp * p->npix;
    for (int k0 = 0; k0 < p->nmaps; k0 += p->chunk) {
        int nm = std::min(p->chunk, p->nmaps - k0);
        if ((rc = use_width(p, nm))) return rc;
        FftArgs f = fft_args(p, nm);
        f.maps_in = map + k0 * mstride;
        {
            StageTimer t(p, SHT_STAGE_FFT_FWD);
            HIPCHK(launch_fft_forward(f, p->classes.data(), (int)p->classes.size(), p->ncomp, p->stream));
        }
        double* a = alm + k0 * astride;
        if ((rc = run_m2a(p, a, nm, 0))) return rc;
        // the rows of T, E and iB are laid out once for both syntheses
        if ((rc = run_to_mmajor(p, a, nm, SHT_COMP_ALL))) return rc;
        if ((rc = run_leg_a2m(p, SHT_COMP_T | SHT_COMP_E))) return rc;
        if ((rc = run_fft_inv(p, map_e + k0 * mstride, nm, SHT_COMP_T | SHT_COMP_E))) return rc;
        if ((rc = run_leg_a2m(p, SHT_COMP_B))) return rc;
        if ((rc = run_fft_inv(p, map_b + k0 * mstride, nm, SHT_COMP_B))) return rc;
    }
    return SHT_OK;
}

int sht_map2alm_iter(sht_plan p, const double* map, double* alm, int niter, double* resid)
{
    int rc = check_ready(p);
    if (rc) return rc;
    if ((rc = whole_only(p, "the iteration"))) return rc;
    if (!alm || !map) return fail(SHT_ERR_ARG, "null data pointer");
    if (niter < 0) return fail(SHT_ERR_ARG, "niter must be >= 0");
    if ((rc = prep(p))) return rc;
    if ((rc = ensure_iter_buffers(p))) return rc;
    const int64_t astride = (int64_t)p->ncomp * (p->lmax + 1) * (p->lmax + 1);
    const int64_t mstride = (int64_t)p->ncomp * p->npix;
    std::vector<double> sums(niter + 1, 0.0), hn;
    for (int k0 = 0; k0 < p->nmaps; k0 += p->chunk) {
        int nm = std::min(p->chunk, p->nmaps - k0);
        if ((rc = use_width(p, nm))) return rc;
        double* a = alm + k0 * astride;
        FftArgs f = fft_args(p, nm);
        f.maps_in = map + k0 * mstride;
        f.F = p->F;
        {
            StageTimer t(p, SHT_STAGE_FFT_FWD);
            HIPCHK(launch_fft_forward(f, p->classes.data(), (int)p->classes.size(), p->ncomp, p->stream));
        }
        if ((rc = run_m2a(p, a, nm, 0))) return rc;
        const int rounds = niter + (resid ? 1 : 0);
        for (int it = 1; it <= rounds; ++it) {
            if ((rc = run_a2m(p, a, nm))) return rc;
            FftArgs r = fft_args(p, nm);
            r.F = p->F;
            r.norms = resid ? p->norms : nullptr;
            r.iteration_sub = (it <= niter);
            if (resid) HIPCHK(hipMemsetAsync(p->norms, 0, (size_t)nm * p->ncomp * sizeof(double), p->stream));
            {
                StageTimer t(p, SHT_STAGE_RESIDUAL);
                HIPCHK(launch_residual(r, p->classes.data(), (int)p->classes.size(), p->ncomp, p->stream));
            }
            if (resid) {
                hn.resize((size_t)nm * p->ncomp);
                HIPCHK(hipMemcpyAsync(hn.data(), p->norms, hn.size() * sizeof(double), hipMemcpyDeviceToHost, p->stream));
                HIPCHK(hipStreamSynchronize(p->stream));
                for (double v : hn) sums[it - 1] += v;
            }
            if (it <= niter)
                if ((rc = run_m2a(p, a, nm, 1))) return rc;
        }
    }
    if (resid) {
        double cnt = (double)p->nmaps * p->ncomp * (double)p->npix;
        for (int n = 0; n <= niter; ++n) resid[n] = std::sqrt(sums[n] / cnt);
    }
    return SHT_OK;
}

int sht_map2alm_immediate(sht_plan p, const double* map, double* alm, int niter, double* resid)
{
    int rc = check_ready(p);
    if (rc) return rc;
    if ((rc = whole_only(p, "the immediate iteration"))) return rc;
    if (!alm || !map) return fail(SHT_ERR_ARG, "null data pointer");
    if (niter < 0) return fail(SHT_ERR_ARG, "niter must be >= 0");
    if ((rc = prep(p))) return rc;
    if ((rc = ensure_iter_buffers(p))) return rc;
    if ((rc = build_levels(p))) return rc;
    if (!p->R || p->R_bytes < p->F_bytes) {
        if (p->R) (void)hipFree(p->R);
        p->R = nullptr;
        HIPCHK(hipMalloc((void**)&p->R, p->F_bytes));
        p->R_bytes = p->F_bytes;
    }
    const int64_t astride = (int64_t)p->ncomp * (p->lmax + 1) * (p->lmax + 1);
    const int64_t mstride = (int64_t)p->ncomp * p->npix;
    const int depth = (int)p->lev.len.size();
    std::vector<double> sums(niter + 1, 0.0), hn;
    auto collect = [&](int n, int nm) -> int {
        hn.resize((size_t)nm * p->ncomp);
        HIPCHK(hipMemcpyAsync(hn.data(), p->norms, hn.size() * sizeof(double), hipMemcpyDeviceToHost, p->stream));
        HIPCHK(hipStreamSynchronize(p->stream));
        for (double v : hn) sums[n] += v;
        return SHT_OK;
    };
    for (int k0 = 0; k0 < p->nmaps; k0 += p->chunk) {
        int nm = std::min(p->chunk, p->nmaps - k0);
        if ((rc = use_width(p, nm))) return rc;
        double* a = alm + k0 * astride;
        FftArgs f = fft_args(p, nm);
        f.maps_in = map + k0 * mstride;
        f.F = p->F;
        {
            StageTimer t(p, SHT_STAGE_FFT_FWD);
            HIPCHK(launch_fft_forward(f, p->classes.data(), (int)p->classes.size(), p->ncomp, p->stream));
        }
        if ((rc = run_m2a(p, a, nm, 0))) return rc;
        if (niter == 0 && !resid) continue;
        // residual spectra of the first estimate, R = F - n C
        if ((rc = run_a2m(p, a, nm))) return rc;
        FftArgs r = fft_args(p, nm);
        r.F = p->F;
        r.R = p->R;
        r.store_res = 1;
        r.norms = resid ? p->norms : nullptr;
        if (resid) HIPCHK(hipMemsetAsync(p->norms, 0, (size_t)nm * p->ncomp * sizeof(double), p->stream));
        {
            StageTimer t(p, SHT_STAGE_RESIDUAL);
            HIPCHK(launch_residual(r, p->classes.data(), (int)p->classes.size(), p->ncomp, p->stream));
        }
        if (resid && (rc = collect(0, nm))) return rc;
        for (int it = 1; it <= niter; ++it) {
            for (int d = 0; d < depth; ++d)
                if ((rc = run_level(p, a, nm, d))) return rc;
            if (resid) {
                HIPCHK(hipMemsetAsync(p->norms, 0, (size_t)nm * p->ncomp * sizeof(double), p->stream));
                FftArgs q = fft_args(p, nm);
                q.R = p->R;
                q.norms = p->norms;
                HIPCHK(launch_hc_norms(q, p->ncomp, p->stream));
                if ((rc = collect(it, nm))) return rc;
            }
        }
    }
    if (resid) {
        double cnt = (double)p->nmaps * p->ncomp * (double)p->npix;
        for (int n = 0; n <= niter; ++n) resid[n] = std::sqrt(sums[n] / cnt);
    }
    return SHT_OK;
}

int sht_plan_set_profiling(sht_plan p, int enable)
{
    if (!p) return fail(SHT_ERR_ARG, "null plan");
    p->profiling = (enable != 0);
    return SHT_OK;
}

int sht_plan_get_profile(sht_plan p, double* ms, long long* launches, int reset)
{
    if (!p) return fail(SHT_ERR_ARG, "null plan");
    if (!ms || !launches) return fail(SHT_ERR_ARG, "null output array");
    HIPCHK(hipStreamSynchronize(p->stream));
    for (int i = 0; i < SHT_NSTAGE; ++i) { ms[i] = 0.0; launches[i] = 0; }
    for (auto& r : p->recs) {
        float t = 0.0f;
        HIPCHK(hipEventElapsedTime(&t, r.a, r.b));
        ms[r.stage] += t;
        launches[r.stage] += 1;
    }
    if (reset) drop_records(p);
    return SHT_OK;
}

int sht_plan_sync(sht_plan p)
{
    if (!p) return fail(SHT_ERR_ARG, "null plan");
    HIPCHK(hipStreamSynchronize(p->stream));
    HIPCHK(hipGetLastError());
    return SHT_OK;
}

}  // extern "C"
