"""Shared test helpers: error measures, tolerances and field construction.

Errors are normwise (the paper checks outputs against naive versions with a
relative error bound, Sec. VII-A; pointwise relative error is undefined near
zero): max|x - ref| / max|ref| and RMS(x - ref) / RMS(ref)."""
import numpy as np

DT = 10.0
SEED = 200513014

# Normwise tolerances: FP64 must agree with the FP64 oracle to 1e-12; FP32
# storage/arithmetic (with FP64 Thomas) to 1e-5; bfloat16 storage carries its
# own output rounding of up to 2^-8 relative, plus the FP32 arithmetic.
TOL = {"f64": 1e-12, "f32": 1e-5, "bf16": 2.0 ** -8 + 1e-5}


def normwise(x, ref):
    """max|x - ref| / max|ref|; an all-zero reference makes it the absolute error."""
    if not x.size:
        return 0.0
    den = np.abs(ref).max()
    err = np.abs(x - ref).max()
    return float(err / den) if den > 0 else float(err)


def rms_rel(x, ref):
    if not x.size:
        return 0.0
    den = np.sqrt(np.mean(ref ** 2))
    err = np.sqrt(np.mean((x - ref) ** 2))
    return float(err / den) if den > 0 else float(err)


def interior(a, h):
    return a if h == 0 else a[:, h:-h, h:-h]


def gpu_fields(f, halo, dtype, names):
    """Device fields (binding.Field) holding the padded arrays f[name]."""
    from paper_2005_13014_amd import binding as B
    return {n: B.Field.from_numpy(f[n], halo, dtype) for n in names}


def out_field(ni, nj, nk, halo, dtype, canary=-7.0):
    """An output field whose halo (and interior) start at a canary value."""
    from paper_2005_13014_amd import binding as B
    return B.Field.empty(ni, nj, nk, halo, dtype, fill=canary)


def halo_untouched(field, canary=-7.0):
    """Every element of the field's allocation outside its interior (halo,
    row and plane padding, alignment slack) still holds the canary."""
    buf = field.buf.detach().to("cpu").double().numpy()
    mask = np.ones(buf.shape, bool)
    k, j, i = np.meshgrid(np.arange(field.nk), np.arange(field.nj), np.arange(field.ni), indexing="ij")
    mask[field.origin + i + field.sj * j + field.sk * k] = False
    return bool(np.all(buf[mask] == canary))


def limiter_masks(u_padded, h, storage):
    """Keep masks (1 = flux kept) of the limiter evaluated in the kernels'
    arithmetic for `storage`: float32 for f32/bf16, float64 for f64.  The
    Laplacian and the fluxes are formed in the order the operator defines,
    which single float32 operations reproduce exactly.  Returns (kx, ky) as
    uint8 arrays with halo 1 in the oracle's flux layout."""
    ft = np.float64 if storage == "f64" else np.float32
    u = u_padded.astype(ft)
    nk, pj, pi = u.shape
    ni, nj = pi - 2 * h, pj - 2 * h

    def U(di, dj):  # u shifted, on the lap domain [-1, ni] x [-1, nj]
        return u[:, h - 1 + dj:h + nj + 1 + dj, h - 1 + di:h + ni + 1 + di]

    four = ft(4)
    lap = four * U(0, 0) - U(1, 0) - U(-1, 0) - U(0, 1) - U(0, -1)   # index [k, j+1, i+1]
    uc = U(0, 0)
    kx = np.zeros((nk, nj + 2, ni + 2), np.uint8)
    ky = np.zeros((nk, nj + 2, ni + 2), np.uint8)
    # x faces i in [-1, ni-1], j in [0, nj)
    f = lap[:, 1:nj + 1, 1:ni + 2] - lap[:, 1:nj + 1, 0:ni + 1]
    du = uc[:, 1:nj + 1, 1:ni + 2] - uc[:, 1:nj + 1, 0:ni + 1]
    kx[:, 1:nj + 1, 0:ni + 1] = ~(f * du > 0)
    f = lap[:, 1:nj + 2, 1:ni + 1] - lap[:, 0:nj + 1, 1:ni + 1]
    du = uc[:, 1:nj + 2, 1:ni + 1] - uc[:, 0:nj + 1, 1:ni + 1]
    ky[:, 0:nj + 1, 1:ni + 1] = ~(f * du > 0)
    return kx, ky
