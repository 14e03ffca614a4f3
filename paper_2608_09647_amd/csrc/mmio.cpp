// Matrix Market reader (Section 3.2: Matrix Market input converted to CSR,
// symmetric storage expanded to the full matrix).  Host code only.
//
// The file is memory-mapped; the entry lines are cut into one contiguous
// chunk per thread at line boundaries and parsed in parallel; the chunks'
// entries are then taken in file order to build CSR with a counting pass,
// a stable scatter (a symmetric file's mirrored entry right after its
// original), a per-row sort by column that keeps file order among equal
// columns, and a merge that sums entries at the same position in that order.
#include <fcntl.h>
#include <omp.h>
#include <sys/mman.h>
#include <sys/stat.h>
#include <unistd.h>

#include <algorithm>
#include <cctype>
#include <climits>
#include <cstdlib>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/cgmi_io.h"
#include "cgmi_host.h"

using cgmi::fail;

namespace {

struct Mapped {
    const char *p = nullptr;
    size_t size = 0;
    int fd = -1;
    ~Mapped() {
        if (p && size) munmap(const_cast<char *>(p), size);
        if (fd >= 0) close(fd);
    }
};

// Line number (1-based) of byte offset off.
int64_t line_of(const char *base, size_t off) {
    return 1 + (int64_t)std::count(base, base + off, '\n');
}

bool is_blank(const char *s, const char *e) {
    for (; s < e; ++s)
        if (!std::isspace((unsigned char)*s)) return false;
    return true;
}

struct Entry {
    int32_t i, j;   // 0-based
    double v;
};

// Parse entry lines in [s, e).  Returns the offset of the first bad line
// (relative to base) or SIZE_MAX.
size_t parse_chunk(const char *base, const char *s, const char *e, int32_t n, bool pattern,
                   std::vector<Entry> &out, std::string &why) {
    char buf[256];
    while (s < e) {
        const char *nl = static_cast<const char *>(memchr(s, '\n', (size_t)(e - s)));
        const char *le = nl ? nl : e;
        if (!is_blank(s, le) && *s != '%') {
            const size_t len = (size_t)(le - s);
            if (len >= sizeof buf) { why = "line too long"; return (size_t)(s - base); }
            std::memcpy(buf, s, len);
            buf[len] = '\0';
            char *q = buf, *r = nullptr;
            const long long i = std::strtoll(q, &r, 10);
            if (r == q) { why = "missing row index"; return (size_t)(s - base); }
            q = r;
            const long long j = std::strtoll(q, &r, 10);
            if (r == q) { why = "missing column index"; return (size_t)(s - base); }
            q = r;
            double v = 1.0;
            if (!pattern) {
                v = std::strtod(q, &r);
                if (r == q) { why = "missing value"; return (size_t)(s - base); }
                q = r;
            }
            while (*q && std::isspace((unsigned char)*q)) ++q;
            if (*q) { why = "trailing characters"; return (size_t)(s - base); }
            if (i < 1 || i > n || j < 1 || j > n) { why = "index out of range"; return (size_t)(s - base); }
            out.push_back(Entry{(int32_t)(i - 1), (int32_t)(j - 1), v});
        }
        s = nl ? nl + 1 : e;
    }
    return SIZE_MAX;
}

std::string lower(std::string s) {
    for (auto &c : s) c = (char)std::tolower((unsigned char)c);
    return s;
}

}  // namespace

extern "C" void cg_mm_free(cg_mm_matrix *m) {
    if (!m) return;
    std::free(m->row_ptr);
    std::free(m->col);
    std::free(m->val);
    std::memset(m, 0, sizeof *m);
}

extern "C" int cg_mm_read(const char *path, int32_t threads, cg_mm_matrix *out) {
    cgmi::clear_error();
    if (!path || !out) return fail(CG_EINVAL, "NULL argument");
    std::memset(out, 0, sizeof *out);
    if (threads < 0) return fail(CG_EINVAL, "threads must be >= 0");
    Mapped f;
    f.fd = open(path, O_RDONLY);
    if (f.fd < 0) return fail(CG_EINVAL, "cannot open %s", path);
    struct stat sb;
    if (fstat(f.fd, &sb) != 0 || sb.st_size <= 0) return fail(CG_EINVAL, "%s: empty or unreadable", path);
    f.size = (size_t)sb.st_size;
    void *mp = mmap(nullptr, f.size, PROT_READ, MAP_PRIVATE, f.fd, 0);
    if (mp == MAP_FAILED) { f.size = 0; return fail(CG_EINVAL, "%s: cannot map the file", path); }
    f.p = static_cast<const char *>(mp);
    const char *base = f.p, *end = f.p + f.size;

    // header line
    bool pattern = false;
    const char *s = base;
    const char *nl = static_cast<const char *>(memchr(s, '\n', f.size));
    {
        std::string h(s, nl ? nl : end);
        char t[5][64] = {};
        const int got = std::sscanf(h.c_str(), "%63s %63s %63s %63s %63s", t[0], t[1], t[2], t[3], t[4]);
        if (got != 5 || lower(t[0]) != "%%matrixmarket" || lower(t[1]) != "matrix")
            return fail(CG_EINVAL, "%s:1: not a Matrix Market matrix header", path);
        const std::string fmt = lower(t[2]), field = lower(t[3]), sym = lower(t[4]);
        if (fmt != "coordinate") return fail(CG_EINVAL, "%s:1: only the coordinate format is read", path);
        if (field != "real" && field != "integer" && field != "pattern")
            return fail(CG_EINVAL, "%s:1: field '%s' not supported (real, integer, pattern)", path, t[3]);
        if (sym != "general" && sym != "symmetric")
            return fail(CG_EINVAL, "%s:1: symmetry '%s' not supported (general, symmetric)", path, t[4]);
        out->symmetric = sym == "symmetric";
        pattern = field == "pattern";
    }
    // comments, then the size line
    s = nl ? nl + 1 : end;
    long long M = -1, N = -1, L = -1;
    while (s < end) {
        nl = static_cast<const char *>(memchr(s, '\n', (size_t)(end - s)));
        const char *le = nl ? nl : end;
        if (*s != '%' && !is_blank(s, le)) {
            std::string line(s, le);
            char extra[8];
            if (std::sscanf(line.c_str(), "%lld %lld %lld %7s", &M, &N, &L, extra) != 3)
                return fail(CG_EINVAL, "%s:%lld: malformed size line", path, (long long)line_of(base, s - base));
            s = nl ? nl + 1 : end;
            break;
        }
        s = nl ? nl + 1 : end;
    }
    if (M < 0) return fail(CG_EINVAL, "%s: no size line", path);
    if (M != N) return fail(CG_EINVAL, "%s: matrix is %lld x %lld, not square", path, M, N);
    if (M > INT32_MAX - 1 || L < 0) return fail(CG_EINVAL, "%s: sizes out of range", path);
    const int32_t n = (int32_t)M;

    // entry lines: one contiguous chunk per thread, cut after a newline
    int T = threads > 0 ? threads : omp_get_max_threads();
    const size_t body = (size_t)(end - s);
    T = (int)std::max<size_t>(1, std::min<size_t>((size_t)T, body / 4096 + 1));
    std::vector<const char *> cut((size_t)T + 1);
    cut[0] = s;
    cut[(size_t)T] = end;
    for (int t = 1; t < T; ++t) {
        const char *c = s + body * (size_t)t / (size_t)T;
        if (c < cut[(size_t)t - 1]) c = cut[(size_t)t - 1];
        const char *q = static_cast<const char *>(memchr(c, '\n', (size_t)(end - c)));
        cut[(size_t)t] = q ? q + 1 : end;
    }
    std::vector<std::vector<Entry>> part((size_t)T);
    std::vector<size_t> bad((size_t)T, SIZE_MAX);
    std::vector<std::string> why((size_t)T);
    bool oom = false;
#pragma omp parallel for num_threads(T) schedule(static, 1)
    for (int t = 0; t < T; ++t) {
        try {
            part[(size_t)t].reserve((size_t)(L / T + 16));
            bad[(size_t)t] = parse_chunk(base, cut[(size_t)t], cut[(size_t)t + 1], n, pattern, part[(size_t)t],
                                         why[(size_t)t]);
        } catch (...) {
#pragma omp atomic write
            oom = true;
        }
    }
    if (oom) return fail(CG_ENOMEM, "out of host memory reading %s", path);
    for (int t = 0; t < T; ++t)
        if (bad[(size_t)t] != SIZE_MAX)
            return fail(CG_EINVAL, "%s:%lld: %s", path, (long long)line_of(base, bad[(size_t)t]),
                        why[(size_t)t].c_str());
    int64_t got = 0;
    for (auto &p : part) got += (int64_t)p.size();
    if (got != L) return fail(CG_EINVAL, "%s: size line announces %lld entries, file holds %lld", path, L,
                              (long long)got);
    out->file_entries = got;

    // expanded entry count per row
    std::vector<int64_t> cnt((size_t)n + 1, 0);
    for (auto &p : part)
        for (const Entry &e : p) {
            ++cnt[(size_t)e.i + 1];
            if (out->symmetric && e.i != e.j) ++cnt[(size_t)e.j + 1];
        }
    for (int32_t i = 0; i < n; ++i) cnt[(size_t)i + 1] += cnt[(size_t)i];
    const int64_t total = cnt[(size_t)n];
    if (total > INT32_MAX) return fail(CG_EINVAL, "%s: %lld stored entries exceed int32 indexing", path,
                                       (long long)total);
    // stable scatter in file order
    std::vector<int32_t> col;
    std::vector<double> val;
    std::vector<int64_t> pos;
    try {
        col.resize((size_t)total);
        val.resize((size_t)total);
        pos.assign(cnt.begin(), cnt.end() - 1);
    } catch (...) {
        return fail(CG_ENOMEM, "out of host memory reading %s", path);
    }
    for (auto &p : part) {
        for (const Entry &e : p) {
            int64_t k = pos[(size_t)e.i]++;
            col[(size_t)k] = e.j;
            val[(size_t)k] = e.v;
            if (out->symmetric && e.i != e.j) {
                k = pos[(size_t)e.j]++;
                col[(size_t)k] = e.i;
                val[(size_t)k] = e.v;
            }
        }
        std::vector<Entry>().swap(p);
    }
    // per row: sort by column keeping file order, sum equal columns in order
    std::vector<int32_t> rlen((size_t)n, 0);
#pragma omp parallel num_threads(T)
    {
        std::vector<std::pair<int32_t, int32_t>> key;   // (column, position in file order)
        std::vector<double> tmp;
#pragma omp for schedule(dynamic, 1024)
        for (int32_t i = 0; i < n; ++i) {
            const int64_t b = cnt[(size_t)i], e = cnt[(size_t)i + 1];
            const int32_t len = (int32_t)(e - b);
            key.resize((size_t)len);
            tmp.assign(val.begin() + b, val.begin() + e);
            for (int32_t k = 0; k < len; ++k) key[(size_t)k] = {col[(size_t)(b + k)], k};
            std::sort(key.begin(), key.end());
            int32_t w = 0;
            for (int32_t k = 0; k < len; ++k) {
                const double v = tmp[(size_t)key[(size_t)k].second];
                if (w > 0 && col[(size_t)(b + w - 1)] == key[(size_t)k].first) {
                    val[(size_t)(b + w - 1)] += v;
                } else {
                    col[(size_t)(b + w)] = key[(size_t)k].first;
                    val[(size_t)(b + w)] = v;
                    ++w;
                }
            }
            rlen[(size_t)i] = w;
        }
    }
    // compact into the caller's arrays
    int64_t nnz = 0;
    for (int32_t i = 0; i < n; ++i) nnz += rlen[(size_t)i];
    out->row_ptr = static_cast<int32_t *>(std::malloc(sizeof(int32_t) * ((size_t)n + 1)));
    out->col = static_cast<int32_t *>(std::malloc(sizeof(int32_t) * (size_t)std::max<int64_t>(nnz, 1)));
    out->val = static_cast<double *>(std::malloc(sizeof(double) * (size_t)std::max<int64_t>(nnz, 1)));
    if (!out->row_ptr || !out->col || !out->val) {
        cg_mm_free(out);
        return fail(CG_ENOMEM, "out of host memory reading %s", path);
    }
    out->row_ptr[0] = 0;
    for (int32_t i = 0; i < n; ++i) out->row_ptr[i + 1] = out->row_ptr[i] + rlen[(size_t)i];
#pragma omp parallel for num_threads(T) schedule(static)
    for (int32_t i = 0; i < n; ++i) {
        const int64_t src = cnt[(size_t)i];
        const int32_t dst = out->row_ptr[i];
        std::memcpy(out->col + dst, col.data() + src, sizeof(int32_t) * (size_t)rlen[(size_t)i]);
        std::memcpy(out->val + dst, val.data() + src, sizeof(double) * (size_t)rlen[(size_t)i]);
    }
    out->n = n;
    out->nnz = nnz;
    return CG_OK;
}
