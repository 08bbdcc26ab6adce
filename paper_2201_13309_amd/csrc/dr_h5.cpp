// HDF5 file layer: per-step image files in, depth-resolved images out.
// Positioned reads for contiguous unfiltered datasets (several threads), the
// HDF5 library for every other layout.
#include "dr_h5.h"

#include <fcntl.h>
#include <hdf5.h>
#include <unistd.h>

#include <algorithm>
#include <atomic>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

namespace {

thread_local std::string g_err;

dr_status fail(dr_status code, const std::string& msg)
{
    g_err = msg;
    return code;
}

dr_status ok()
{
    g_err.clear();
    return DR_OK;
}

// Silence the library's own error printing once per process.
void quiet()
{
    static std::once_flag f;
    std::call_once(f, [] { H5Eset_auto2(H5E_DEFAULT, nullptr, nullptr); });
}

// Closes an HDF5 identifier with the matching call when it leaves scope.
struct Id {
    hid_t id = -1;
    herr_t (*close)(hid_t) = nullptr;
    Id(hid_t i, herr_t (*c)(hid_t)) : id(i), close(c) {}
    ~Id()
    {
        if (id >= 0 && close) close(id);
    }
    Id(const Id&) = delete;
    Id& operator=(const Id&) = delete;
    operator hid_t() const { return id; }
    bool bad() const { return id < 0; }
};

struct FileInfo {
    std::string path;
    int64_t offset = -1;  // byte offset of a contiguous unfiltered dataset, or -1
};

// Link creation that makes missing intermediate groups ("/entry1/data/data").
hid_t make_lcpl()
{
    const hid_t l = H5Pcreate(H5P_LINK_CREATE);
    if (l >= 0) H5Pset_create_intermediate_group(l, 1);
    return l;
}

}  // namespace

struct dr_h5_stack_s {
    std::vector<FileInfo> files;
    std::string dataset;
    int32_t ny = 0, nx = 0, rank = 2;
    int32_t direct = 0;
};

namespace {

// Shape and storage of `dataset` in `path`; rank 2 [ny][nx] or rank 3 [1][ny][nx].
dr_status inspect(const std::string& path, const std::string& dataset, int32_t* ny, int32_t* nx,
                  int32_t* rank, int64_t* offset)
{
    Id f(H5Fopen(path.c_str(), H5F_ACC_RDONLY, H5P_DEFAULT), H5Fclose);
    if (f.bad()) return fail(DR_E_INVAL, "cannot open " + path);
    Id d(H5Dopen2(f, dataset.c_str(), H5P_DEFAULT), H5Dclose);
    if (d.bad()) return fail(DR_E_INVAL, "no dataset " + dataset + " in " + path);
    Id t(H5Dget_type(d), H5Tclose);
    if (t.bad() || H5Tget_class(t) != H5T_INTEGER || H5Tget_size(t) != 2 ||
        H5Tget_sign(t) != H5T_SGN_NONE)
        return fail(DR_E_INVAL, dataset + " in " + path + " is not unsigned 16-bit");
    Id sp(H5Dget_space(d), H5Sclose);
    hsize_t dims[3] = {0, 0, 0};
    const int r = H5Sget_simple_extent_ndims(sp);
    if (r != 2 && r != 3) return fail(DR_E_INVAL, dataset + " in " + path + " is not an image");
    H5Sget_simple_extent_dims(sp, dims, nullptr);
    if (r == 3 && dims[0] != 1)
        return fail(DR_E_INVAL, dataset + " in " + path + " holds more than one image");
    *rank = r;
    *ny = (int32_t)dims[r - 2];
    *nx = (int32_t)dims[r - 1];
    *offset = -1;
    Id pl(H5Dget_create_plist(d), H5Pclose);
    const bool le = H5Tget_order(t) == H5T_ORDER_LE;
    if (!pl.bad() && le && H5Pget_layout(pl) == H5D_CONTIGUOUS && H5Pget_nfilters(pl) == 0) {
        const haddr_t a = H5Dget_offset(d);
        if (a != HADDR_UNDEF) *offset = (int64_t)a;
    }
    return DR_OK;
}

// Rows [row0, row0 + nrows) of one file through the library.
dr_status read_library(const dr_h5_stack_s& s, const FileInfo& fi, int32_t row0, int32_t nrows,
                       uint16_t* out)
{
    Id f(H5Fopen(fi.path.c_str(), H5F_ACC_RDONLY, H5P_DEFAULT), H5Fclose);
    if (f.bad()) return fail(DR_E_DEVICE, "cannot open " + fi.path);
    Id d(H5Dopen2(f, s.dataset.c_str(), H5P_DEFAULT), H5Dclose);
    if (d.bad()) return fail(DR_E_DEVICE, "cannot open " + s.dataset + " in " + fi.path);
    Id sp(H5Dget_space(d), H5Sclose);
    hsize_t start[3] = {0, 0, 0}, count[3] = {1, 1, 1};
    const int r = s.rank;
    start[r - 2] = (hsize_t)row0;
    count[r - 2] = (hsize_t)nrows;
    count[r - 1] = (hsize_t)s.nx;
    if (H5Sselect_hyperslab(sp, H5S_SELECT_SET, start, nullptr, count, nullptr) < 0)
        return fail(DR_E_DEVICE, "row selection failed in " + fi.path);
    const hsize_t mdims[1] = {(hsize_t)nrows * (hsize_t)s.nx};
    Id ms(H5Screate_simple(1, mdims, nullptr), H5Sclose);
    if (H5Dread(d, H5T_NATIVE_USHORT, ms, sp, H5P_DEFAULT, out) < 0)
        return fail(DR_E_DEVICE, "read failed in " + fi.path);
    return DR_OK;
}

// The same rows by positioned reads at the dataset's byte offset.
dr_status read_direct(const dr_h5_stack_s& s, const FileInfo& fi, int32_t row0, int32_t nrows,
                      uint16_t* out)
{
    const int fd = ::open(fi.path.c_str(), O_RDONLY);
    if (fd < 0) return fail(DR_E_DEVICE, "cannot open " + fi.path);
    const size_t bytes = (size_t)nrows * (size_t)s.nx * sizeof(uint16_t);
    off_t pos = (off_t)fi.offset + (off_t)row0 * s.nx * (off_t)sizeof(uint16_t);
    char* dst = reinterpret_cast<char*>(out);
    size_t done = 0;
    while (done < bytes) {
        const ssize_t r = ::pread(fd, dst + done, bytes - done, pos + (off_t)done);
        if (r <= 0) break;
        done += (size_t)r;
    }
    ::close(fd);
    if (done != bytes) return fail(DR_E_DEVICE, "short read in " + fi.path);
    return DR_OK;
}

}  // namespace

extern "C" {

const char* dr_h5_last_error(void) { return g_err.c_str(); }

dr_status dr_h5_open_stack(const char* const* paths, int32_t n_files, const char* dataset,
                           dr_h5_stack* out)
{
    if (!paths || !dataset || !out || n_files < 1)
        return fail(DR_E_INVAL, "dr_h5_open_stack: bad argument");
    *out = nullptr;
    quiet();
    auto s = std::make_unique<dr_h5_stack_s>();
    s->dataset = dataset;
    s->files.resize((size_t)n_files);
    for (int32_t k = 0; k < n_files; ++k) {
        if (!paths[k]) return fail(DR_E_INVAL, "dr_h5_open_stack: NULL path");
        FileInfo& fi = s->files[(size_t)k];
        fi.path = paths[k];
        int32_t ny = 0, nx = 0, rank = 2;
        dr_status st = inspect(fi.path, s->dataset, &ny, &nx, &rank, &fi.offset);
        if (st != DR_OK) return st;
        if (k == 0) {
            s->ny = ny;
            s->nx = nx;
            s->rank = rank;
        } else if (ny != s->ny || nx != s->nx || rank != s->rank) {
            return fail(DR_E_INVAL, "image shape of " + fi.path + " differs from the first file");
        }
        if (fi.offset >= 0) s->direct++;
    }
    if (s->ny < 1 || s->nx < 1) return fail(DR_E_INVAL, "empty images");
    *out = s.release();
    return ok();
}

dr_status dr_h5_stack_shape(dr_h5_stack s, int32_t* n_files, int32_t* ny, int32_t* nx,
                            int32_t* direct_files)
{
    if (!s) return fail(DR_E_INVAL, "dr_h5_stack_shape: NULL stack");
    if (n_files) *n_files = (int32_t)s->files.size();
    if (ny) *ny = s->ny;
    if (nx) *nx = s->nx;
    if (direct_files) *direct_files = s->direct;
    return ok();
}

dr_status dr_h5_read_rows(dr_h5_stack s, int32_t row0, int32_t nrows, uint16_t* out,
                          int32_t nthreads)
{
    if (!s || !out) return fail(DR_E_INVAL, "dr_h5_read_rows: NULL argument");
    if (row0 < 0 || nrows < 1 || row0 + nrows > s->ny)
        return fail(DR_E_INVAL, "dr_h5_read_rows: rows outside the image");
    const int64_t n = (int64_t)s->files.size();
    const size_t per = (size_t)nrows * (size_t)s->nx;
    // files read through the library first, on this thread (the library
    // serialises its calls); the rest by positioned reads on a pool
    for (int64_t k = 0; k < n; ++k)
        if (s->files[(size_t)k].offset < 0) {
            dr_status st = read_library(*s, s->files[(size_t)k], row0, nrows, out + (size_t)k * per);
            if (st != DR_OK) return st;
        }
    const int T = (int)std::max<int64_t>(1, std::min<int64_t>(nthreads > 0 ? nthreads : 16, n));
    std::atomic<int64_t> next{0};
    std::atomic<int> failed{0};
    std::mutex mu;
    std::string first_err;
    auto work = [&]() {
        for (;;) {
            const int64_t k = next.fetch_add(1);
            if (k >= n || failed.load()) return;
            const FileInfo& fi = s->files[(size_t)k];
            if (fi.offset < 0) continue;
            if (read_direct(*s, fi, row0, nrows, out + (size_t)k * per) != DR_OK) {
                std::lock_guard<std::mutex> lk(mu);
                if (!failed.exchange(1)) first_err = g_err;
            }
        }
    };
    std::vector<std::thread> pool;
    for (int t = 1; t < T; ++t) pool.emplace_back(work);
    work();
    for (auto& th : pool) th.join();
    if (failed.load()) return fail(DR_E_DEVICE, first_err);
    return ok();
}

dr_status dr_h5_close_stack(dr_h5_stack s)
{
    if (!s) return fail(DR_E_INVAL, "dr_h5_close_stack: NULL stack");
    delete s;
    return ok();
}

dr_status dr_h5_read_scalars(const char* const* paths, int32_t n_files, const char* dataset,
                             double* out)
{
    if (!paths || !dataset || !out || n_files < 0)
        return fail(DR_E_INVAL, "dr_h5_read_scalars: bad argument");
    quiet();
    for (int32_t k = 0; k < n_files; ++k) {
        if (!paths[k]) return fail(DR_E_INVAL, "dr_h5_read_scalars: NULL path");
        Id f(H5Fopen(paths[k], H5F_ACC_RDONLY, H5P_DEFAULT), H5Fclose);
        if (f.bad()) return fail(DR_E_INVAL, std::string("cannot open ") + paths[k]);
        Id d(H5Dopen2(f, dataset, H5P_DEFAULT), H5Dclose);
        if (d.bad()) return fail(DR_E_INVAL, std::string("no dataset ") + dataset + " in " + paths[k]);
        Id sp(H5Dget_space(d), H5Sclose);
        if (H5Sget_simple_extent_npoints(sp) != 1)
            return fail(DR_E_INVAL, std::string(dataset) + " is not a scalar in " + paths[k]);
        if (H5Dread(d, H5T_NATIVE_DOUBLE, H5S_ALL, H5S_ALL, H5P_DEFAULT, out + k) < 0)
            return fail(DR_E_INVAL, std::string(dataset) + " is not numeric in " + paths[k]);
    }
    return ok();
}

dr_status dr_h5_write_stack(const char* const* paths, int32_t n_files, const char* dataset,
                            const uint16_t* images, int32_t ny, int32_t nx, int32_t deflate_level)
{
    if (!paths || !dataset || !images || n_files < 1 || ny < 1 || nx < 1 || deflate_level < 0 ||
        deflate_level > 9)
        return fail(DR_E_INVAL, "dr_h5_write_stack: bad argument");
    quiet();
    const hsize_t dims[2] = {(hsize_t)ny, (hsize_t)nx};
    for (int32_t k = 0; k < n_files; ++k) {
        if (!paths[k]) return fail(DR_E_INVAL, "dr_h5_write_stack: NULL path");
        Id f(H5Fcreate(paths[k], H5F_ACC_TRUNC, H5P_DEFAULT, H5P_DEFAULT), H5Fclose);
        if (f.bad()) return fail(DR_E_INVAL, std::string("cannot create ") + paths[k]);
        Id sp(H5Screate_simple(2, dims, nullptr), H5Sclose);
        Id pl(H5Pcreate(H5P_DATASET_CREATE), H5Pclose);
        if (deflate_level > 0) {
            const hsize_t chunk[2] = {(hsize_t)std::min(64, ny), (hsize_t)nx};
            H5Pset_chunk(pl, 2, chunk);
            H5Pset_deflate(pl, (unsigned)deflate_level);
        }
        Id lc(make_lcpl(), H5Pclose);
        Id d(H5Dcreate2(f, dataset, H5T_STD_U16LE, sp, lc, pl, H5P_DEFAULT), H5Dclose);
        if (d.bad()) return fail(DR_E_INVAL, std::string("cannot create ") + dataset);
        if (H5Dwrite(d, H5T_NATIVE_USHORT, H5S_ALL, H5S_ALL, H5P_DEFAULT,
                     images + (size_t)k * (size_t)ny * (size_t)nx) < 0)
            return fail(DR_E_DEVICE, std::string("write failed: ") + paths[k]);
    }
    return ok();
}

dr_status dr_h5_write_scalars(const char* const* paths, int32_t n_files, const char* dataset,
                              const double* values)
{
    if (!paths || !dataset || !values || n_files < 0)
        return fail(DR_E_INVAL, "dr_h5_write_scalars: bad argument");
    quiet();
    for (int32_t k = 0; k < n_files; ++k) {
        if (!paths[k]) return fail(DR_E_INVAL, "dr_h5_write_scalars: NULL path");
        Id f(H5Fopen(paths[k], H5F_ACC_RDWR, H5P_DEFAULT), H5Fclose);
        if (f.bad()) return fail(DR_E_INVAL, std::string("cannot open ") + paths[k]);
        Id sp(H5Screate(H5S_SCALAR), H5Sclose);
        Id lc(make_lcpl(), H5Pclose);
        Id d(H5Dcreate2(f, dataset, H5T_IEEE_F64LE, sp, lc, H5P_DEFAULT, H5P_DEFAULT), H5Dclose);
        if (d.bad()) return fail(DR_E_INVAL, std::string("cannot create ") + dataset);
        if (H5Dwrite(d, H5T_NATIVE_DOUBLE, H5S_ALL, H5S_ALL, H5P_DEFAULT, values + k) < 0)
            return fail(DR_E_DEVICE, std::string("write failed: ") + paths[k]);
    }
    return ok();
}

dr_status dr_h5_write_depth_images(const char* path, const char* dataset, const float* images,
                                   int32_t n_bins, int32_t ny, int32_t nx, double first_center,
                                   double width)
{
    if (!path || !dataset || !images || n_bins < 1 || ny < 1 || nx < 1)
        return fail(DR_E_INVAL, "dr_h5_write_depth_images: bad argument");
    quiet();
    Id f(H5Fcreate(path, H5F_ACC_TRUNC, H5P_DEFAULT, H5P_DEFAULT), H5Fclose);
    if (f.bad()) return fail(DR_E_INVAL, std::string("cannot create ") + path);
    const hsize_t dims[3] = {(hsize_t)n_bins, (hsize_t)ny, (hsize_t)nx};
    Id sp(H5Screate_simple(3, dims, nullptr), H5Sclose);
    Id lc(make_lcpl(), H5Pclose);
    Id d(H5Dcreate2(f, dataset, H5T_IEEE_F32LE, sp, lc, H5P_DEFAULT, H5P_DEFAULT), H5Dclose);
    if (d.bad()) return fail(DR_E_INVAL, std::string("cannot create ") + dataset);
    if (H5Dwrite(d, H5T_NATIVE_FLOAT, H5S_ALL, H5S_ALL, H5P_DEFAULT, images) < 0)
        return fail(DR_E_DEVICE, std::string("write failed: ") + path);
    std::vector<double> depth((size_t)n_bins);
    for (int32_t b = 0; b < n_bins; ++b) depth[(size_t)b] = first_center + b * width;
    const hsize_t bd[1] = {(hsize_t)n_bins};
    Id sp1(H5Screate_simple(1, bd, nullptr), H5Sclose);
    const std::string dname = std::string(dataset) + "_depth";
    Id d1(H5Dcreate2(f, dname.c_str(), H5T_IEEE_F64LE, sp1, lc, H5P_DEFAULT, H5P_DEFAULT),
          H5Dclose);
    if (d1.bad()) return fail(DR_E_INVAL, "cannot create " + dname);
    if (H5Dwrite(d1, H5T_NATIVE_DOUBLE, H5S_ALL, H5S_ALL, H5P_DEFAULT, depth.data()) < 0)
        return fail(DR_E_DEVICE, std::string("write failed: ") + path);
    return ok();
}

}  // extern "C"
