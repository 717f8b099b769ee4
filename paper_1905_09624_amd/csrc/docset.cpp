// Document front-end: files in the formats the paper reads (section 2.3:
// DNA FASTA files, multi-document FASTA files, text files) turned into the
// string/document layout of cobs_docs.  Reads (FASTA records, FASTQ reads)
// are separate strings, so no q-gram spans two of them; a text file is one
// continuous string.  Host only.
#include <cstdio>
#include <string>
#include <vector>

#include "runtime.h"

using namespace cobs;

struct cobs_docset {
    std::vector<uint8_t> bytes;
    std::vector<uint64_t> str_off{0};   // string s = bytes[str_off[s], str_off[s+1])
    std::vector<uint64_t> doc_str{0};   // document d = strings [doc_str[d], doc_str[d+1])
};

namespace {

bool is_space(uint8_t c) { return c == ' ' || c == '\t' || c == '\r' || c == '\n' || c == '\v' || c == '\f'; }

void end_string(cobs_docset *ds) { ds->str_off.push_back(ds->bytes.size()); }
void end_document(cobs_docset *ds) { ds->doc_str.push_back(ds->str_off.size() - 1); }

// Lines of [p, p + n) without their line terminator ("\n" or "\r\n").
template <typename F>
void for_lines(const uint8_t *p, uint64_t n, F f)
{
    uint64_t a = 0;
    while (a < n) {
        uint64_t b = a;
        while (b < n && p[b] != '\n') ++b;
        uint64_t e = b;
        if (e > a && p[e - 1] == '\r') --e;
        f(p + a, e - a);
        a = b + 1;
    }
}

// FASTA: a record is a '>' header line and the sequence lines up to the next
// header; ';' lines are comments; whitespace inside sequence lines is dropped.
// per_record: one document per record, else one document for the file.
cobs_status parse_fasta(cobs_docset *ds, const uint8_t *p, uint64_t n, bool per_record)
{
    bool open = false;
    for_lines(p, n, [&](const uint8_t *l, uint64_t len) {
        if (len && l[0] == '>') {
            if (open) {
                end_string(ds);
                if (per_record) end_document(ds);
            }
            open = true;
            return;
        }
        if (len && l[0] == ';') return;
        if (!open) {
            bool blank = true;
            for (uint64_t i = 0; i < len; ++i) blank &= is_space(l[i]);
            if (blank) return;
            open = true;   // sequence before any header: one record
        }
        for (uint64_t i = 0; i < len; ++i)
            if (!is_space(l[i])) ds->bytes.push_back(l[i]);
    });
    if (open) {
        end_string(ds);
        if (per_record) end_document(ds);
    }
    if (!per_record) end_document(ds);
    return COBS_OK;
}

// FASTQ: four-line records ('@' header, sequence, '+' line, quality of the
// sequence's length); blank lines between records are skipped.
cobs_status parse_fastq(cobs_docset *ds, const uint8_t *p, uint64_t n)
{
    std::vector<std::pair<const uint8_t *, uint64_t>> lines;
    for_lines(p, n, [&](const uint8_t *l, uint64_t len) { lines.emplace_back(l, len); });
    const size_t str0 = ds->str_off.size(), byte0 = ds->bytes.size();
    size_t i = 0;
    while (i < lines.size()) {
        if (lines[i].second == 0) { ++i; continue; }
        if (i + 3 >= lines.size()) {
            ds->str_off.resize(str0);
            ds->bytes.resize(byte0);
            return set_error(COBS_EINVAL, "FASTQ record " + std::to_string(i / 4) + " is truncated");
        }
        const auto &h = lines[i], &s = lines[i + 1], &plus = lines[i + 2], &q = lines[i + 3];
        if (h.first[0] != '@' || plus.second == 0 || plus.first[0] != '+' || q.second != s.second) {
            ds->str_off.resize(str0);
            ds->bytes.resize(byte0);
            return set_error(COBS_EINVAL, "malformed FASTQ record at line " + std::to_string(i + 1));
        }
        ds->bytes.insert(ds->bytes.end(), s.first, s.first + s.second);
        end_string(ds);
        i += 4;
    }
    end_document(ds);
    return COBS_OK;
}

cobs_status add(cobs_docset *ds, const uint8_t *p, uint64_t n, uint32_t format)
{
    switch (format) {
    case COBS_FORMAT_FASTA: return parse_fasta(ds, p, n, false);
    case COBS_FORMAT_MULTI_FASTA: return parse_fasta(ds, p, n, true);
    case COBS_FORMAT_FASTQ: return parse_fastq(ds, p, n);
    case COBS_FORMAT_TEXT:
        ds->bytes.insert(ds->bytes.end(), p, p + n);
        end_string(ds);
        end_document(ds);
        return COBS_OK;
    default: return set_error(COBS_EINVAL, "unknown document format");
    }
}

}  // namespace

extern "C" {

cobs_status cobs_docset_create(cobs_docset **out)
{
    if (!out) return set_error(COBS_EINVAL, "NULL argument");
    *out = new cobs_docset();
    return COBS_OK;
}

cobs_status cobs_docset_add_buffer(cobs_docset *ds, const uint8_t *data, uint64_t len, uint32_t format)
{
    if (!ds || (len && !data)) return set_error(COBS_EINVAL, "NULL argument");
    return add(ds, data, len, format);
}

cobs_status cobs_docset_add_file(cobs_docset *ds, const char *path, uint32_t format)
{
    if (!ds || !path) return set_error(COBS_EINVAL, "NULL argument");
    FILE *f = std::fopen(path, "rb");
    if (!f) return set_error(COBS_EINVAL, std::string("cannot open ") + path);
    std::vector<uint8_t> buf;
    uint8_t chunk[1 << 16];
    size_t got;
    while ((got = std::fread(chunk, 1, sizeof chunk, f)) > 0) buf.insert(buf.end(), chunk, chunk + got);
    const bool err = std::ferror(f) != 0;
    std::fclose(f);
    if (err) return set_error(COBS_EINVAL, std::string("read failed: ") + path);
    return add(ds, buf.data(), buf.size(), format);
}

cobs_status cobs_docset_view(const cobs_docset *ds, cobs_docs *docs)
{
    if (!ds || !docs) return set_error(COBS_EINVAL, "NULL argument");
    docs->bytes = ds->bytes.data();
    docs->str_off = ds->str_off.data();
    docs->doc_str = ds->doc_str.data();
    docs->n_docs = (uint32_t)(ds->doc_str.size() - 1);
    docs->mem = COBS_MEM_HOST;
    return COBS_OK;
}

void cobs_docset_free(cobs_docset *ds) { delete ds; }

}  // extern "C"
