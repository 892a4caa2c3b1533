// line_io.cpp -- the "Input" task of the pipeline (§3.5): line records of
// the HITRAN fixed-width format (160 characters per record) read into the
// arrays hk_load_lines and hk_opacity_stream take.  Host code only.
#include "../../include/hk.h"

#include <algorithm>
#include <cerrno>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

namespace hk {
void set_thread_error(const char* msg);  // the message hk_last_error(NULL) returns
}

namespace {

int io_fail(const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    hk::set_thread_error(buf);
    return HK_EINVAL;
}

constexpr int kRecord = 160;

struct Field {
    const char* name;
    int col, width;  // 1-based first column, characters
};
// Fortran edit descriptors of the layout: I2 I1 F12.6 E10.3 E10.3 F5.4 F5.3
// F10.4 F4.2 F8.6 ...
constexpr Field kMol{"molecule", 1, 2};
constexpr Field kNu{"nu", 4, 12};
constexpr Field kS{"S_ref", 16, 10};
constexpr Field kA{"A21", 26, 10};
constexpr Field kGair{"gamma_air", 36, 5};
constexpr Field kGself{"gamma_self", 41, 5};
constexpr Field kE{"E_lower", 46, 10};
constexpr Field kN{"n_air", 56, 4};
constexpr Field kD{"delta", 60, 8};

// The number in a fixed-width field: blanks around it, nothing else.
bool parse(const char* rec, const Field& f, double* v)
{
    char buf[32];
    std::memcpy(buf, rec + f.col - 1, (size_t)f.width);
    buf[f.width] = '\0';
    char* p = buf;
    while (*p == ' ') ++p;
    if (!*p) return false;
    errno = 0;
    char* end = nullptr;
    *v = std::strtod(p, &end);
    if (end == p || errno == ERANGE) return false;
    while (*end == ' ') ++end;
    return *end == '\0';
}

struct File {
    FILE* f = nullptr;
    ~File()
    {
        if (f) std::fclose(f);
    }
};

}  // namespace

extern "C" int hk_read_par(const char* path, int64_t first, int32_t molecule, const hk_lines_out* out,
                           int64_t* n_read, int64_t* next)
{
    if (!path || !out || !n_read || !next) return io_fail("path, out, n_read and next must not be NULL");
    *n_read = 0;
    *next = first;
    if (first < 0) return io_fail("first = %lld must be >= 0", (long long)first);
    if (molecule < 0 || molecule > 99) return io_fail("molecule = %d out of [0, 99]", molecule);
    if (out->capacity < 0) return io_fail("capacity = %lld must be >= 0", (long long)out->capacity);
    if (out->capacity > 0 && (!out->nu || !out->S_ref || !out->E_lower || !out->gamma_air || !out->n_air ||
                              !out->gamma_self || !out->delta || !out->A21))
        return io_fail("every output array is required");
    File fh;
    fh.f = std::fopen(path, "rb");
    if (!fh.f) return io_fail("cannot open %s: %s", path, std::strerror(errno));
    // record length from the first record's line end: LF or CR LF
    char head[kRecord + 2];
    const size_t got = std::fread(head, 1, sizeof head, fh.f);
    if (got == 0) return HK_OK;  // an empty file holds no records
    int reclen = 0;
    if (got >= kRecord + 1 && head[kRecord] == '\n')
        reclen = kRecord + 1;
    else if (got == kRecord + 2 && head[kRecord] == '\r' && head[kRecord + 1] == '\n')
        reclen = kRecord + 2;
    else
        return io_fail("%s: the first record is not 160 characters and a line end", path);
    if (std::fseek(fh.f, 0, SEEK_END) != 0) return io_fail("%s: cannot seek", path);
    const long size = std::ftell(fh.f);
    if (size < 0) return io_fail("%s: cannot tell its size", path);
    const int64_t n_rec = (int64_t)size / reclen;
    if ((int64_t)size % reclen != 0)
        return io_fail("%s: record %lld is truncated (%ld bytes is not a whole number of %d-byte records)", path,
                       (long long)n_rec, size, reclen);
    if (first >= n_rec) {
        *next = n_rec;
        return HK_OK;
    }
    if (std::fseek(fh.f, (long)(first * reclen), SEEK_SET) != 0) return io_fail("%s: cannot seek", path);
    const int64_t block = 4096;
    std::vector<char> buf((size_t)(block * reclen));
    int64_t rec = first, stored = 0;
    while (rec < n_rec && stored < out->capacity) {
        const int64_t want = std::min<int64_t>(block, n_rec - rec);
        if (std::fread(buf.data(), (size_t)reclen, (size_t)want, fh.f) != (size_t)want)
            return io_fail("%s: read error at record %lld", path, (long long)rec);
        for (int64_t k = 0; k < want && stored < out->capacity; ++k, ++rec) {
            const char* r = buf.data() + k * reclen;
            if (r[reclen - 1] != '\n' || (reclen == kRecord + 2 && r[kRecord] != '\r'))
                return io_fail("%s: record %lld does not end after 160 characters", path, (long long)rec);
            double v[9];
            const Field* fs[9] = {&kMol, &kNu, &kS, &kA, &kGair, &kGself, &kE, &kN, &kD};
            if (!parse(r, kMol, &v[0])) return io_fail("%s: record %lld: field molecule", path, (long long)rec);
            if (molecule > 0 && (int)v[0] != molecule) continue;
            for (int q = 1; q < 9; ++q)
                if (!parse(r, *fs[q], &v[q]))
                    return io_fail("%s: record %lld: field %s (columns %d-%d)", path, (long long)rec, fs[q]->name,
                                   fs[q]->col, fs[q]->col + fs[q]->width - 1);
            out->nu[stored] = v[1];
            out->S_ref[stored] = v[2];
            out->A21[stored] = v[3];
            out->gamma_air[stored] = v[4];
            out->gamma_self[stored] = v[5];
            out->E_lower[stored] = v[6];
            out->n_air[stored] = v[7];
            out->delta[stored] = v[8];
            ++stored;
        }
    }
    *n_read = stored;
    *next = rec;
    return HK_OK;
}
