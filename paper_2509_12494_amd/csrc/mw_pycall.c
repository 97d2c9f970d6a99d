/* Direct-call shim for the Python binding (mwntt.py), argument marshalling
 * only.  The binding passes the addresses of six entry points of libmwntt
 * (taken from its ctypes handle) to bind() once; each call then converts
 * plain integer arguments and calls the entry point with the GIL released,
 * exactly as a ctypes call would, at a fraction of ctypes' per-call cost.
 * No computation of the library happens here, and the library itself stays
 * the only code that touches the device.
 *
 *   bind(ntt_forward, ntt_inverse, vec_addmod, vec_submod, vec_mulmod, vec_axpymod)
 *   ntt(direction, plan, d_out, d_in, batch, stream)          -> status
 *   blas(op, d_c, d_a, d_b, n, q_words, limbs, stream)         -> status (op 0 add, 1 sub, 2 mul)
 *   axpy(d_y, alpha_words, d_x, n, q_words, limbs, stream)     -> status
 *
 * Pointers are Python ints (0 or None for NULL); q_words / alpha_words are
 * addresses of host arrays of 64-bit words that the caller keeps alive for
 * the duration of the call.  Statuses are the library's (mwntt.h). */
#define PY_SSIZE_T_CLEAN
#include <Python.h>
#include <stddef.h>
#include <stdint.h>

typedef int (*ntt_fn)(void*, void*, const void*, uint32_t, void*);
typedef int (*bin_fn)(void*, const void*, const void*, size_t, const uint64_t*, uint32_t, void*);
typedef int (*axpy_fn)(void*, const uint64_t*, const void*, size_t, const uint64_t*, uint32_t, void*);

static ntt_fn g_ntt[2];
static bin_fn g_bin[3];
static axpy_fn g_axpy;

static int get_ptr(PyObject* o, void** out) {
  if (o == Py_None) {
    *out = NULL;
    return 0;
  }
  void* p = PyLong_AsVoidPtr(o);
  if (p == NULL && PyErr_Occurred()) return -1;
  *out = p;
  return 0;
}

static int get_u64(PyObject* o, unsigned long long* out) {
  const unsigned long long v = PyLong_AsUnsignedLongLong(o);
  if (v == (unsigned long long)-1 && PyErr_Occurred()) return -1;
  *out = v;
  return 0;
}

static int nargs_is(Py_ssize_t nargs, Py_ssize_t want, const char* name) {
  if (nargs == want) return 1;
  PyErr_Format(PyExc_TypeError, "%s takes %zd arguments (%zd given)", name, want, nargs);
  return 0;
}

static PyObject* bind(PyObject* self, PyObject* const* args, Py_ssize_t nargs) {
  (void)self;
  void* p[6];
  if (!nargs_is(nargs, 6, "bind")) return NULL;
  for (int i = 0; i < 6; ++i) {
    if (get_ptr(args[i], &p[i])) return NULL;
    if (!p[i]) {
      PyErr_SetString(PyExc_ValueError, "bind: null entry point");
      return NULL;
    }
  }
  g_ntt[0] = (ntt_fn)p[0];
  g_ntt[1] = (ntt_fn)p[1];
  g_bin[0] = (bin_fn)p[2];
  g_bin[1] = (bin_fn)p[3];
  g_bin[2] = (bin_fn)p[4];
  g_axpy = (axpy_fn)p[5];
  Py_RETURN_NONE;
}

static PyObject* ntt(PyObject* self, PyObject* const* args, Py_ssize_t nargs) {
  (void)self;
  unsigned long long dir, batch;
  void *plan, *out, *in, *stream;
  if (!nargs_is(nargs, 6, "ntt")) return NULL;
  if (get_u64(args[0], &dir) || get_ptr(args[1], &plan) || get_ptr(args[2], &out) || get_ptr(args[3], &in) ||
      get_u64(args[4], &batch) || get_ptr(args[5], &stream))
    return NULL;
  if (dir > 1 || batch > UINT32_MAX) {
    PyErr_SetString(PyExc_ValueError, "ntt: direction must be 0 or 1 and batch below 2^32");
    return NULL;
  }
  const ntt_fn f = g_ntt[dir];
  if (!f) {
    PyErr_SetString(PyExc_RuntimeError, "ntt: entry points not bound");
    return NULL;
  }
  int st;
  Py_BEGIN_ALLOW_THREADS
  st = f(plan, out, in, (uint32_t)batch, stream);
  Py_END_ALLOW_THREADS
  return PyLong_FromLong(st);
}

static PyObject* blas(PyObject* self, PyObject* const* args, Py_ssize_t nargs) {
  (void)self;
  unsigned long long op, n, limbs;
  void *c, *a, *b, *q, *stream;
  if (!nargs_is(nargs, 8, "blas")) return NULL;
  if (get_u64(args[0], &op) || get_ptr(args[1], &c) || get_ptr(args[2], &a) || get_ptr(args[3], &b) ||
      get_u64(args[4], &n) || get_ptr(args[5], &q) || get_u64(args[6], &limbs) || get_ptr(args[7], &stream))
    return NULL;
  if (op > 2 || limbs > UINT32_MAX) {
    PyErr_SetString(PyExc_ValueError, "blas: op must be 0, 1 or 2");
    return NULL;
  }
  const bin_fn f = g_bin[op];
  if (!f) {
    PyErr_SetString(PyExc_RuntimeError, "blas: entry points not bound");
    return NULL;
  }
  int st;
  Py_BEGIN_ALLOW_THREADS
  st = f(c, a, b, (size_t)n, (const uint64_t*)q, (uint32_t)limbs, stream);
  Py_END_ALLOW_THREADS
  return PyLong_FromLong(st);
}

static PyObject* axpy(PyObject* self, PyObject* const* args, Py_ssize_t nargs) {
  (void)self;
  unsigned long long n, limbs;
  void *y, *alpha, *x, *q, *stream;
  if (!nargs_is(nargs, 7, "axpy")) return NULL;
  if (get_ptr(args[0], &y) || get_ptr(args[1], &alpha) || get_ptr(args[2], &x) || get_u64(args[3], &n) ||
      get_ptr(args[4], &q) || get_u64(args[5], &limbs) || get_ptr(args[6], &stream))
    return NULL;
  if (limbs > UINT32_MAX) {
    PyErr_SetString(PyExc_ValueError, "axpy: argument out of range");
    return NULL;
  }
  if (!g_axpy) {
    PyErr_SetString(PyExc_RuntimeError, "axpy: entry points not bound");
    return NULL;
  }
  int st;
  Py_BEGIN_ALLOW_THREADS
  st = g_axpy(y, (const uint64_t*)alpha, x, (size_t)n, (const uint64_t*)q, (uint32_t)limbs, stream);
  Py_END_ALLOW_THREADS
  return PyLong_FromLong(st);
}

static PyMethodDef methods[] = {
    {"bind", (PyCFunction)(void (*)(void))bind, METH_FASTCALL, "bind the six entry point addresses"},
    {"ntt", (PyCFunction)(void (*)(void))ntt, METH_FASTCALL, "ntt_forward / ntt_inverse"},
    {"blas", (PyCFunction)(void (*)(void))blas, METH_FASTCALL, "vec_addmod / vec_submod / vec_mulmod"},
    {"axpy", (PyCFunction)(void (*)(void))axpy, METH_FASTCALL, "vec_axpymod"},
    {NULL, NULL, 0, NULL}};

static struct PyModuleDef module = {PyModuleDef_HEAD_INIT, "_mwcall", "direct calls into libmwntt", -1, methods,
                                    NULL, NULL, NULL, NULL};

PyMODINIT_FUNC PyInit__mwcall(void) { return PyModule_Create(&module); }
